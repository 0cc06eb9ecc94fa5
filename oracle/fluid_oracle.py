"""FP64 numpy oracle of the fluid step of the operator-split reactive Euler solver (Le & Cambier,
arXiv:1110.4903, Sec. 3.1 with the governing equations of Sec. 2).

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the HIP library or its binding.
Written for clarity, not speed: whole-array numpy operations, no fusion.

What it computes, for a 2-D grid of cells holding the conserved variables of Sec. 2,
Q = (rho_s [Ns], rho u, rho v, E) with E = sum_s rho_s e_s + rho |u|^2 / 2:

  - the mixture thermodynamics of NASA-7 species: the energy e_s each species carries on the
    fluid side leaves out its formation energy (Sec. 2, Eq. energy), here
    e_s(T) = e_s^NASA(T) - e_s^NASA(T_ref) with T_ref = 298.15 K, so that the chemistry sub-step
    of the split (the library's conserved-variable adapter) sees the same energy; the pressure is
    Dalton's law P = sum_s rho_s (R / M_s) T (Sec. 2, Eq. dalton), the temperature the root of
    sum_s rho_s e_s(T) = E - rho |u|^2 / 2, and the sound speed c^2 = gamma P / rho with the
    frozen ratio gamma = c_p / c_v of the mixture;
  - MP5 reconstruction (Sec. 3.1, Eq. mp5) of the primitive variables (rho_s, u_n, u_t, P) at
    every cell face, each limited by the monotonicity-preserving bound of Eqs. mp and ump
    (alpha = 2);
  - the HLLE flux (Sec. 3.1, Eq. fluxhlle) with the wave-speed bounds b+ and b- built from the
    outer states' speeds and a Roe-type average;
  - third-order Runge-Kutta time integration of each one-dimensional sweep;
  - dimensional splitting: a step is an x sweep then a y sweep (or the reverse order).

Readings of points the paper leaves open or prints garbled (listed with the design notes):
  - the printed HLLE formula has F_L and F_R exchanged against the upwind limit (with b- = 0 it
    would return the downstream flux); the flux taken is the standard one,
    F = (b+ F_L - b- F_R) / (b+ - b-) + b+ b- / (b+ - b-) (Q_R - Q_L);
  - the averaged normal velocity and sound speed of b+-: the square-root-density average of
    u_n and Einfeldt's average of c^2 plus his velocity-jump term, which needs no assumption on
    the equation of state;
  - MP5 acts on the primitive variables (rho_s, u_n, u_t, P), component by component; the
    right state of a face is the mirror image of the left state's formula and limiter;
  - the Runge-Kutta scheme is the three-stage strong-stability-preserving one of Shu and Osher;
  - three ghost cells per side: periodic, or zero-gradient (transmissive) copies.
"""
from __future__ import annotations

import numpy as np

R_U = 8.31446261815324   # J/(mol K)
T_REF = 298.15
ALPHA_MP = 2.0
NG = 3                   # ghost cells per side


class Gas:
    """NASA-7 mixture thermodynamics, vectorised over cells: arrays are [Ns][...]."""

    def __init__(self, mech):
        self.ns = mech.ns
        self.Mkg = np.asarray(mech.M, np.float64) * 1e-3        # kg/mol
        self.nasa = np.asarray(mech.nasa, np.float64)           # [ns][2][7]
        self.Tmid = np.asarray(mech.T_mid, np.float64)
        self.Rs = R_U / self.Mkg                                # J/(kg K)
        self.e_ref = self._e_nasa(np.full(1, T_REF))[:, 0]

    def _coef(self, T):
        """[ns][7][...] coefficients of the set that applies at each T."""
        hi = T[None, ...] >= self.Tmid.reshape((-1,) + (1,) * T.ndim)
        lo = self.nasa[:, 0].reshape(self.ns, 7, *([1] * T.ndim))
        up = self.nasa[:, 1].reshape(self.ns, 7, *([1] * T.ndim))
        return np.where(hi[:, None], up, lo)

    def _e_nasa(self, T):
        """e_s = (R/M_s)(h_s/R - T), h_s/R = a1 T + a2 T^2/2 + a3 T^3/3 + a4 T^4/4 + a5 T^5/5 + a6."""
        a = self._coef(T)
        h = (a[:, 0] * T + a[:, 1] * T ** 2 / 2 + a[:, 2] * T ** 3 / 3 + a[:, 3] * T ** 4 / 4 +
             a[:, 4] * T ** 5 / 5 + a[:, 5])
        return self.Rs.reshape((-1,) + (1,) * T.ndim) * (h - T)

    def e_sens(self, T):
        """Fluid-side species energy e_s(T) - e_s(T_ref), J/kg, [ns][...]."""
        return self._e_nasa(T) - self.e_ref.reshape((-1,) + (1,) * T.ndim)

    def cp_R(self, T):
        a = self._coef(T)
        return a[:, 0] + a[:, 1] * T + a[:, 2] * T ** 2 + a[:, 3] * T ** 3 + a[:, 4] * T ** 4

    def cv(self, rho_s, T):
        """Mixture c_v times density: sum_s rho_s (R/M_s)(cp_s/R - 1), J/(m^3 K)."""
        Rs = self.Rs.reshape((-1,) + (1,) * T.ndim)
        return (rho_s * Rs * (self.cp_R(T) - 1.0)).sum(0)

    def gamma(self, rho_s, T):
        Rs = self.Rs.reshape((-1,) + (1,) * T.ndim)
        cv = self.cv(rho_s, T)
        return (cv + (rho_s * Rs).sum(0)) / cv

    def pressure(self, rho_s, T):
        Rs = self.Rs.reshape((-1,) + (1,) * T.ndim)
        return (rho_s * Rs).sum(0) * T

    def temperature(self, rho_s, e_int, T0=None, iters=60):
        """Root of sum_s rho_s e_s(T) = e_int (J/m^3) by Newton's method on the monotone
        function (d/dT = rho c_v > 0) from T0 (default 1000 K), to |dT| <= 1e-13 T."""
        T = np.full(e_int.shape, 1000.0) if T0 is None else np.array(T0, dtype=np.float64)
        for _ in range(iters):
            f = (rho_s * self.e_sens(T)).sum(0) - e_int
            dT = f / self.cv(rho_s, T)
            T = T - dT
            if np.all(np.abs(dT) <= 1e-13 * np.abs(T)):
                return T
        raise RuntimeError("temperature inversion did not converge")


def to_primitive(gas, Q, T0=None):
    """Q [ns + 3][...] -> W = (rho_s, u, v, P) [ns + 3][...] and T."""
    ns = gas.ns
    rho_s = Q[:ns]
    rho = rho_s.sum(0)
    u, v = Q[ns] / rho, Q[ns + 1] / rho
    T = gas.temperature(rho_s, Q[ns + 2] - 0.5 * rho * (u * u + v * v), T0)
    W = np.concatenate([rho_s, u[None], v[None], gas.pressure(rho_s, T)[None]])
    return W, T


def to_conserved(gas, W):
    """W = (rho_s, u, v, P) -> Q and T (T = P / sum_s rho_s R_s, no inversion)."""
    ns = gas.ns
    rho_s, u, v, P = W[:ns], W[ns], W[ns + 1], W[ns + 2]
    Rs = gas.Rs.reshape((-1,) + (1,) * u.ndim)
    T = P / (rho_s * Rs).sum(0)
    rho = rho_s.sum(0)
    E = (rho_s * gas.e_sens(T)).sum(0) + 0.5 * rho * (u * u + v * v)
    return np.concatenate([rho_s, (rho * u)[None], (rho * v)[None], E[None]]), T


def minmod(a, b):
    return np.where(a * b > 0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


def median(a, b, c):
    return a + minmod(b - a, c - a)


def mp5_left(um2, um1, u0, up1, up2):
    """Left state at face j+1/2 from cells j-2..j+2 (Eq. mp5), limited by Eqs. mp and ump."""
    uL = (2 * um2 - 13 * um1 + 47 * u0 + 27 * up1 - 3 * up2) / 60.0
    ump = u0 + minmod(up1 - u0, ALPHA_MP * (u0 - um1))
    return median(uL, u0, ump)


def mp5_faces(w):
    """Left and right states of every interior face of a ghost-extended row along the last
    axis: w[..., m] with m = n + 2 NG cells gives faces between cells NG-1+k and NG+k,
    k = 0..n (n + 1 faces)."""
    m = w.shape[-1]
    n = m - 2 * NG
    j = np.arange(NG - 1, NG + n)          # the face j + 1/2 for each j
    s = lambda d: w[..., j + d]
    uL = mp5_left(s(-2), s(-1), s(0), s(1), s(2))
    # mirror image: the right state of face j+1/2 from cells j+3..j-1
    uR = mp5_left(s(3), s(2), s(1), s(0), s(-1))
    return uL, uR


def euler_flux(gas, W, Q):
    """Flux along the first velocity component of the state (its normal direction)."""
    ns = gas.ns
    u, P = W[ns], W[ns + 2]
    F = Q * u
    F[ns] = F[ns] + P
    F[ns + 2] = F[ns + 2] + u * P
    return F


def hlle(gas, WL, WR):
    """HLLE flux (Eq. fluxhlle) between left and right primitive states (normal velocity in
    component ns, tangential in ns + 1)."""
    ns = gas.ns
    QL, TL = to_conserved(gas, WL)
    QR, TR = to_conserved(gas, WR)
    rL, rR = WL[:ns].sum(0), WR[:ns].sum(0)
    uL, uR = WL[ns], WR[ns]
    cL = np.sqrt(gas.gamma(WL[:ns], TL) * WL[ns + 2] / rL)
    cR = np.sqrt(gas.gamma(WR[:ns], TR) * WR[ns + 2] / rR)
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    u_hat = (sL * uL + sR * uR) / (sL + sR)
    c2_hat = (sL * cL ** 2 + sR * cR ** 2) / (sL + sR) + 0.5 * sL * sR / (sL + sR) ** 2 * (uR - uL) ** 2
    c_hat = np.sqrt(c2_hat)
    bp = np.maximum(0.0, np.maximum(u_hat + c_hat, uR + cR))
    bm = np.minimum(0.0, np.minimum(u_hat - c_hat, uL - cL))
    FL, FR = euler_flux(gas, WL, QL), euler_flux(gas, WR, QR)
    return (bp * FL - bm * FR) / (bp - bm) + (bp * bm / (bp - bm)) * (QR - QL)


def _ghost(a, bc):
    """Extend the last axis by NG cells per side."""
    if bc == "periodic":
        if a.shape[-1] < NG:
            raise ValueError("a periodic direction needs at least NG cells")
        return np.concatenate([a[..., -NG:], a, a[..., :NG]], axis=-1)
    if bc == "outflow":
        return np.concatenate([np.repeat(a[..., :1], NG, axis=-1), a, np.repeat(a[..., -1:], NG, axis=-1)], axis=-1)
    raise ValueError(bc)


def sweep_rhs(gas, Q, h, axis, bc, T0=None):
    """-(F_{j+1/2} - F_{j-1/2}) / h along axis (0 = x, the last array axis; 1 = y) of Q
    [ns + 3][ny][nx]."""
    ns = gas.ns
    W, _ = to_primitive(gas, Q, T0)
    if axis == 1:                           # rows become the y direction; u_n = v, u_t = u
        W = np.swapaxes(W, -1, -2)[[*range(ns), ns + 1, ns, ns + 2]]
    WL, WR = mp5_faces(_ghost(W, bc))
    F = hlle(gas, WL, WR)
    dQ = -(F[..., 1:] - F[..., :-1]) / h
    if axis == 1:
        dQ = np.swapaxes(dQ[[*range(ns), ns + 1, ns, ns + 2]], -1, -2)
    return dQ


def rk3_sweep(gas, Q, dt, h, axis, bc):
    """Three-stage strong-stability-preserving Runge-Kutta step of one sweep."""
    Q1 = Q + dt * sweep_rhs(gas, Q, h, axis, bc)
    Q2 = 0.75 * Q + 0.25 * (Q1 + dt * sweep_rhs(gas, Q1, h, axis, bc))
    return Q / 3.0 + 2.0 / 3.0 * (Q2 + dt * sweep_rhs(gas, Q2, h, axis, bc))


def fluid_step(gas, Q, dt, dx, dy, bc="periodic", y_first=False):
    """One dimensionally split step: an x sweep then a y sweep (the reverse with y_first)."""
    if y_first:
        return rk3_sweep(gas, rk3_sweep(gas, Q, dt, dy, 1, bc), dt, dx, 0, bc)
    return rk3_sweep(gas, rk3_sweep(gas, Q, dt, dx, 0, bc), dt, dy, 1, bc)


def max_dt(gas, Q, dx, dy, cfl):
    """cfl times the smallest dx / (|u| + c) and dy / (|v| + c) over the grid."""
    ns = gas.ns
    W, T = to_primitive(gas, Q)
    c = np.sqrt(gas.gamma(W[:ns], T) * W[ns + 2] / W[:ns].sum(0))
    return cfl * min(dx / float(np.max(np.abs(W[ns]) + c)), dy / float(np.max(np.abs(W[ns + 1]) + c)))
