"""ctypes wrapper of the FP64 CPU oracle (kin_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the benchmark's
CPU-baseline leg, never by the HIP library or its binding.  ``build()`` compiles the C
source with gcc (-O2 -fno-fast-math -ffp-contract=off -fopenmp); ``lib()`` builds on first
use if the shared object is missing or older than its sources.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, f) for f in ("kin_oracle.c", "kin_oracle_eval.inc", "kin_oracle.h")]
SO = os.path.join(HERE, "liborc.so")

OK, OK_HALVED, FAILED, BAD_INPUT = 0, 1, 2, 3


def build(force: bool = True) -> str:
    if not force and os.path.exists(SO) and all(os.path.getmtime(SO) >= os.path.getmtime(s) for s in SRC):
        return SO
    tmp = SO + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-Wno-unused-function", "-o", tmp, os.path.join(HERE, "kin_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, SO)
    return SO


class _Mech(C.Structure):
    _fields_ = [("ns", C.c_int), ("nr", C.c_int), ("ntb", C.c_int),
                ("M", C.c_void_p), ("nasa", C.c_void_p), ("T_mid", C.c_void_p),
                ("reac_idx", C.c_void_p), ("reac_nu", C.c_void_p),
                ("prod_idx", C.c_void_p), ("prod_nu", C.c_void_p),
                ("A", C.c_void_p), ("b", C.c_void_p), ("Ta", C.c_void_p),
                ("reversible", C.c_void_p), ("tb", C.c_void_p), ("eff", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol_Y", C.c_double), ("atol_T", C.c_double),
                ("y_neg", C.c_double), ("k_max", C.c_int), ("L_max", C.c_int),
                ("max_iters", C.c_int), ("diverge_ratio", C.c_double), ("point_implicit", C.c_int)]


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        build(force=False)
        L = C.CDLL(SO)
        vp, d, i, l = C.c_void_p, C.c_double, C.c_int, C.c_long
        L.orc_default_opts.argtypes = [vp]
        L.orc_species_thermo.argtypes = [vp, d, vp, vp, vp, vp]
        L.orc_mix_energy.argtypes = [vp, vp, d]; L.orc_mix_energy.restype = d
        L.orc_mix_cv.argtypes = [vp, vp, d]; L.orc_mix_cv.restype = d
        L.orc_rates.argtypes = [vp, d, vp, d, vp, vp, vp, vp, vp, vp, vp]
        L.orc_rhs.argtypes = [vp, d, vp, vp]
        L.orc_jacobian.argtypes = [vp, d, vp, vp]
        L.orc_jacobian_fd.argtypes = [vp, d, vp, vp]
        L.orc_lu_factor.argtypes = [i, vp, vp]; L.orc_lu_factor.restype = i
        L.orc_lu_solve.argtypes = [i, vp, vp, vp]
        L.orc_invert_T.argtypes = [vp, vp, d, d, vp]; L.orc_invert_T.restype = i
        L.orc_be_substep.argtypes = [vp, d, d, vp, d, vp, vp, vp]; L.orc_be_substep.restype = i
        L.orc_advance.argtypes = [vp, l, vp, vp, vp, vp, d, vp, i, vp, vp, vp, vp, i]
        L.orc_follow.argtypes = [vp, l, vp, vp, vp, vp, d, vp, vp, i, vp, vp, vp, vp, i]
        L.orc_energy_batch.argtypes = [vp, l, vp, vp, vp]
        L.orc_residual_ld.argtypes = [vp, d, vp, vp, d, vp, vp]; L.orc_residual_ld.restype = d
        L.orc_term_scale.argtypes = [vp, d, vp, vp, d, vp]
        L.orc_num_threads.restype = i
        _LIB = L
    return _LIB


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def default_opts() -> Opts:
    o = Opts()
    lib().orc_default_opts(C.byref(o))
    return o


def make_opts(rtol=None, atol_Y=None, atol_T=None, y_neg=None, k_max=None, L_max=None,
              max_iters=None, point_implicit=None, diverge_ratio=None) -> Opts:
    o = default_opts()
    for k, v in dict(rtol=rtol, atol_Y=atol_Y, atol_T=atol_T, y_neg=y_neg, k_max=k_max,
                     L_max=L_max, max_iters=max_iters, point_implicit=point_implicit,
                     diverge_ratio=diverge_ratio).items():
        if v is not None:
            setattr(o, k, v)
    return o


# Reference temperature of the fluid side's sensible energy (K): the species formation
# energies it leaves out are e_s(T_REF).
T_REF = 298.15


class OracleMech:
    """Holds contiguous copies of a synth.Mechanism's arrays and the C view of them."""

    def __init__(self, mech):
        self.mech = mech
        self.ns, self.nr = mech.ns, mech.nr
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        self._keep = dict(M=f64(mech.M), nasa=f64(mech.nasa), T_mid=f64(mech.T_mid),
                          reac_idx=i32(mech.reac_idx), reac_nu=i32(mech.reac_nu),
                          prod_idx=i32(mech.prod_idx), prod_nu=i32(mech.prod_nu),
                          A=f64(mech.A), b=f64(mech.b), Ta=f64(mech.Ta),
                          reversible=i32(mech.reversible), tb=i32(mech.tb),
                          eff=f64(mech.eff if mech.eff.size else np.zeros((1, mech.ns))))
        s = _Mech()
        s.ns, s.nr, s.ntb = mech.ns, mech.nr, mech.ntb
        for k, v in self._keep.items():
            setattr(s, k, v.ctypes.data)
        self.c = s
        self.ref = C.byref(self.c)

    # -- species / mixture functions ----------------------------------------------------------
    def thermo(self, T: float):
        out = [np.zeros(self.ns) for _ in range(4)]
        lib().orc_species_thermo(self.ref, float(T), *[_p(a) for a in out])
        return out  # cp/R, h/RT, s/R, d(cp/R)/dT

    def energy(self, Y, T: float) -> float:
        return lib().orc_mix_energy(self.ref, _p(np.ascontiguousarray(Y, np.float64)), float(T))

    def cv(self, Y, T: float) -> float:
        return lib().orc_mix_cv(self.ref, _p(np.ascontiguousarray(Y, np.float64)), float(T))

    def rates(self, rho: float, Y, T: float):
        nr, ns = self.nr, self.ns
        kf, kb, Mc, qf, qb, q = (np.zeros(nr) for _ in range(6))
        wdot = np.zeros(ns)
        lib().orc_rates(self.ref, float(rho), _p(np.ascontiguousarray(Y, np.float64)), float(T),
                        _p(kf), _p(kb), _p(Mc), _p(qf), _p(qb), _p(q), _p(wdot))
        return dict(kf=kf, kb=kb, M=Mc, qf=qf, qb=qb, q=q, wdot=wdot)

    def rhs(self, rho: float, x):
        f = np.zeros(self.ns + 1)
        lib().orc_rhs(self.ref, float(rho), _p(np.ascontiguousarray(x, np.float64)), _p(f))
        return f

    def jacobian(self, rho: float, x, fd: bool = False):
        N = self.ns + 1
        J = np.zeros((N, N))
        fn = lib().orc_jacobian_fd if fd else lib().orc_jacobian
        fn(self.ref, float(rho), _p(np.ascontiguousarray(x, np.float64)), _p(J))
        return J

    def invert_T(self, Y, e0: float, T_start: float):
        T = np.zeros(1)
        rc = lib().orc_invert_T(self.ref, _p(np.ascontiguousarray(Y, np.float64)), float(e0), float(T_start), _p(T))
        return rc, float(T[0])

    def be_substep(self, rho: float, e0: float, x, h: float, opts: Optional[Opts] = None):
        """One sub-step: (rc, x after T inversion, Newton iterations, Newton root)."""
        x = np.array(x, dtype=np.float64)
        xbe = np.zeros_like(x)
        it = np.zeros(1, np.int32)
        rc = lib().orc_be_substep(self.ref, float(rho), float(e0), _p(x), float(h),
                                  C.byref(opts or default_opts()), _p(it), _p(xbe))
        return rc, x, int(it[0]), xbe

    def residual(self, rho: float, x_prev, x, h: float, opts: Optional[Opts] = None):
        G = np.zeros(self.ns + 1)
        w = lib().orc_residual_ld(self.ref, float(rho), _p(np.ascontiguousarray(x_prev, np.float64)),
                                  _p(np.ascontiguousarray(x, np.float64)), float(h),
                                  C.byref(opts or default_opts()), _p(G))
        return w, G

    def term_scale(self, rho: float, Y_prev, x, h: float):
        S = np.zeros(self.ns)
        lib().orc_term_scale(self.ref, float(rho), _p(np.ascontiguousarray(Y_prev, np.float64)),
                             _p(np.ascontiguousarray(x, np.float64)), float(h), _p(S))
        return S

    # -- operator-split adapter (Sec. 2: the energy equation and the operator-splitting
    #    equation; the fluid side's energy leaves out the species formation energies) ---------
    def formation_energies(self):
        """e_s(T_ref) in J/kg at T_ref = 298.15 K: the part of each species' internal energy
        (NASA-7 h with the formation enthalpy, minus RT) that the fluid-side energy leaves out."""
        unit = np.eye(self.ns)
        return np.array([self.energy(unit[s], T_REF) for s in range(self.ns)])

    def from_conserved(self, rho_s, E_sens, T_guess=None):
        """(rho, Y, T, e0, ok) from partial densities rho_s[Ns][n] (kg/m^3) and the sensible
        energy E_sens[n] = sum_s rho_s (e_s(T) - e_s(T_ref)) (J/m^3): rho = sum rho_s,
        Y = rho_s / rho, e0 = E_sens / rho + sum_s Y_s e_s(T_ref), T the root of e(Y, T) = e0
        (Newton from T_guess or 1500 K, then bisection); ok is False (and T NaN) without a root."""
        rho_s = np.asarray(rho_s, np.float64)
        E_sens = np.asarray(E_sens, np.float64)
        n = rho_s.shape[1]
        ef = self.formation_energies()
        rho = rho_s.sum(axis=0)
        Y = rho_s / rho
        e0 = E_sens / rho + ef @ Y
        T = np.full(n, np.nan)
        ok = np.zeros(n, bool)
        for i in range(n):
            start = 1500.0 if T_guess is None else float(T_guess[i])
            if not 200.0 <= start <= 6000.0:
                start = 1500.0
            rc, Ti = self.invert_T(Y[:, i], e0[i], start)
            if rc == 0:
                T[i], ok[i] = Ti, True
        return rho, Y, T, e0, ok

    def to_conserved(self, rho, Y, e0):
        """(rho_s[Ns][n], E_sens[n]) of cells with density rho, mass fractions Y and internal
        energy e0 (formation energies included): rho_s = rho Y, E_sens = rho (e0 - sum Y e_s(T_ref))."""
        ef = self.formation_energies()
        rho = np.asarray(rho, np.float64)
        Y = np.asarray(Y, np.float64)
        return rho * Y, rho * (np.asarray(e0, np.float64) - ef @ Y)

    # -- batch ------------------------------------------------------------------------------
    def energy_batch(self, T, Y):
        T = np.ascontiguousarray(T, np.float64)
        Y = np.ascontiguousarray(Y, np.float64)
        e0 = np.zeros(T.shape[0])
        lib().orc_energy_batch(self.ref, T.shape[0], _p(T), _p(Y), _p(e0))
        return e0

    def advance(self, rho, T, Y, dt: float, e0=None, opts: Optional[Opts] = None, L_forced: int = -1,
                nthreads: int = 0, with_sched: bool = False):
        """Advance cells one dt; returns (T, Y, status, level, iters[, sched]) as new arrays."""
        rho = np.ascontiguousarray(rho, np.float64)
        n = rho.shape[0]
        T = np.array(T, dtype=np.float64)
        Y = np.array(Y, dtype=np.float64).reshape(self.ns, n)
        e0p = None if e0 is None else np.ascontiguousarray(e0, np.float64)
        st, lv, it = (np.zeros(n, np.int32) for _ in range(3))
        sh = np.zeros(n, np.uint64)
        lib().orc_advance(self.ref, n, _p(rho), None if e0p is None else _p(e0p), _p(T), _p(Y),
                          float(dt), C.byref(opts or default_opts()), int(L_forced),
                          _p(st), _p(lv), _p(it), _p(sh), int(nthreads))
        if with_sched:
            return T, Y, st, lv, it, sh
        return T, Y, st, lv, it

    def follow(self, rho, T, Y, dt: float, e0, trace, opts: Optional[Opts] = None, nthreads: int = 0):
        """Advance cells along given sub-step schedules (trace[n][words]: word 0 the attempt
        count, then the accept bits); returns (T, Y, status, level, iters, sched) as new arrays.
        status -1: an attempt the schedule accepts does not converge here; -2: schedule
        truncated."""
        rho = np.ascontiguousarray(rho, np.float64)
        n = rho.shape[0]
        T = np.array(T, dtype=np.float64)
        Y = np.array(Y, dtype=np.float64).reshape(self.ns, n)
        e0 = np.ascontiguousarray(e0, np.float64)
        trace = np.ascontiguousarray(trace, np.uint64)
        assert trace.ndim == 2 and trace.shape[0] == n
        st, lv, it = (np.zeros(n, np.int32) for _ in range(3))
        sh = np.zeros(n, np.uint64)
        lib().orc_follow(self.ref, n, _p(rho), _p(e0), _p(T), _p(Y), float(dt), C.byref(opts or default_opts()),
                         _p(trace), int(trace.shape[1]), _p(st), _p(lv), _p(it), _p(sh), int(nthreads))
        return T, Y, st, lv, it, sh


def lu_factor(A):
    A = np.array(A, dtype=np.float64)
    n = A.shape[0]
    piv = np.zeros(n, np.int32)
    rc = lib().orc_lu_factor(n, _p(A), _p(piv))
    return rc, A, piv


def lu_solve(LU, piv, b):
    b = np.array(b, dtype=np.float64)
    lib().orc_lu_solve(LU.shape[0], _p(np.ascontiguousarray(LU)), _p(np.ascontiguousarray(piv, np.int32)), _p(b))
    return b


def num_threads() -> int:
    return lib().orc_num_threads()
