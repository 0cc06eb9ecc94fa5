"""Seeded synthetic mechanisms and cell states.

This module only *generates inputs*: element compositions, reaction lists found by
search over those compositions, Arrhenius parameters, NASA-7 coefficient sets and
cell states.  It evaluates none of the kinetics (no rates, no thermodynamic
functions of T, no Jacobians); both the FP64 CPU oracle and the HIP library take
its arrays as plain inputs.

Why synthetic: the paper lists the 19 reversible H2-air reaction equations of its
9-species case (Appendix A) but prints no Arrhenius or thermodynamic data, and its
36-species/308-reaction hydrocarbon mechanism is only named (Sec. 5.2).  The
generator therefore builds mechanisms with the same species and reaction counts
(9 species / 38 reactions and 36 species / 308 reactions, Sec. 5.2) and the same
reaction templates as Appendix A: exchange reactions A+B <=> C+D and third-body
combinations A+B(+M) <=> C, element-balanced over seeded compositions.

Every random draw comes from ``numpy.random.default_rng(seed)`` in a fixed order,
so a (recipe, seed) pair always yields bit-identical arrays.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from collections import defaultdict
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# Standard atomic weights (g/mol) of the elements the synthetic species are built from.
ELEMENT_MASS = {"H": 1.008, "O": 15.999, "N": 14.007, "C": 12.011, "S": 32.06}
ELEMENT_ORDER = ("H", "O", "N", "C", "S")

# NASA-7 fit interval used for every synthetic species (K).
T_FIT_LO, T_FIT_MID, T_FIT_HI = 300.0, 1000.0, 5000.0
T_REF = 298.15

MAX_SLOTS = 3  # reactant / product entries per reaction (index, stoichiometric coefficient)


@dataclasses.dataclass
class Mechanism:
    """Reaction mechanism as flat arrays (the layout both libraries accept).

    Units: molar masses g/mol; Arrhenius ``A`` in CGS (cm^3/mol)^(order-1)/s with the
    third-body concentration counted in the order; ``Ta = E/R`` in K; NASA-7
    coefficients dimensionless (cp/R polynomial in T, a6 in K, a7 dimensionless).
    Reaction entries use species index -1 and coefficient 0 for an empty slot.
    ``tb[r]`` is -1 for a plain reaction, else the row of ``eff`` holding that
    reaction's third-body efficiencies.
    """

    name: str
    elements: Tuple[str, ...]
    comp: np.ndarray        # [Ns][E] int8 atoms per element
    M: np.ndarray           # [Ns] float64
    nasa: np.ndarray        # [Ns][2][7] float64; [:,0,:] used for T < T_mid, [:,1,:] otherwise
    T_lo: np.ndarray        # [Ns]
    T_mid: np.ndarray       # [Ns]
    T_hi: np.ndarray        # [Ns]
    reac_idx: np.ndarray    # [R][3] int32
    reac_nu: np.ndarray     # [R][3] int32
    prod_idx: np.ndarray    # [R][3] int32
    prod_nu: np.ndarray     # [R][3] int32
    A: np.ndarray           # [R] float64
    b: np.ndarray           # [R] float64
    Ta: np.ndarray          # [R] float64
    reversible: np.ndarray  # [R] int32 (1 reversible, 0 irreversible)
    tb: np.ndarray          # [R] int32
    eff: np.ndarray         # [Ntb][Ns] float64

    @property
    def ns(self) -> int:
        return int(self.M.shape[0])

    @property
    def nr(self) -> int:
        return int(self.A.shape[0])

    @property
    def ne(self) -> int:
        return int(self.comp.shape[1])

    @property
    def ntb(self) -> int:
        return int(self.eff.shape[0])

    def save(self, path: str) -> None:
        """Write a round-trip-exact binary file (numpy .npz, no pickled objects)."""
        arrays = {f.name: getattr(self, f.name) for f in dataclasses.fields(self)
                  if isinstance(getattr(self, f.name), np.ndarray)}
        np.savez(path, name=np.array(self.name), elements=np.array(self.elements), **arrays)

    @staticmethod
    def load(path: str) -> "Mechanism":
        with np.load(path, allow_pickle=False) as z:
            kw = {k: z[k] for k in z.files if k not in ("name", "elements")}
            return Mechanism(name=str(z["name"]), elements=tuple(str(e) for e in z["elements"]), **kw)

    def equation(self, r: int) -> str:
        def side(idx, nu):
            parts = []
            for i, n in zip(idx, nu):
                if i >= 0:
                    parts.append(("2 " if n == 2 else "") + f"S{i}")
            return " + ".join(parts)
        m = " (+M)" if self.tb[r] >= 0 else ""
        arrow = " <=> " if self.reversible[r] else " => "
        return side(self.reac_idx[r], self.reac_nu[r]) + m + arrow + side(self.prod_idx[r], self.prod_nu[r]) + m


# ----------------------------------------------------------------------------------------------
# Recipes
# ----------------------------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class MechRecipe:
    name: str
    seed: int
    n_elements: int
    n_species: int
    n_reactions: int
    frac_third_body: float
    frac_irreversible: float
    logA_range: Tuple[float, float] = (8.0, 14.0)      # log10 A, A in cm^3/mol/s (cm^6/mol^2/s for +M)
    b_range: Tuple[float, float] = (-1.5, 1.5)
    Ta_range: Tuple[float, float] = (0.0, 3.0e4)       # K
    eff_range: Tuple[float, float] = (0.5, 3.0)
    cp_range: Tuple[float, float] = (2.5, 8.0)         # cp/R bounds over the fit interval
    hf_bond_R: float = 2.0e4                           # K released per bond formed (see make_mechanism)
    hf_noise_R: float = 5.0e3                          # K, half-width of the uniform hf/R noise
    exothermic_forward: bool = True                    # orient exchange reactions downhill in h


def _round_half_up(x: float) -> int:
    return int(math.floor(x + 0.5))


MECH9 = MechRecipe("mech9", seed=9038, n_elements=3, n_species=9, n_reactions=38,
                   frac_third_body=0.10, frac_irreversible=0.0)
MECH36 = MechRecipe("mech36", seed=36308, n_elements=4, n_species=36, n_reactions=308,
                    frac_third_body=0.15, frac_irreversible=0.30)
RECIPES = {"mech9": MECH9, "mech36": MECH36}


def _candidates(comps: np.ndarray):
    """All element-balanced equations of the two templates over a composition set.

    Combination: A + B -> C with comp(A) + comp(B) = comp(C) (A = B allowed, giving 2A).
    Exchange: A + B -> C + D with equal summed composition and no species on both sides.
    Each equation is listed once (unordered sides, unordered pair of sides).
    """
    ns = comps.shape[0]
    key = {tuple(int(v) for v in c): i for i, c in enumerate(comps)}
    pairs = [(i, j) for i in range(ns) for j in range(i, ns)]
    comb, by_sum = [], defaultdict(list)
    for (i, j) in pairs:
        s = tuple(int(v) for v in comps[i] + comps[j])
        by_sum[s].append((i, j))
        if s in key:
            comb.append((i, j, key[s]))
    exch = []
    for s in sorted(by_sum):
        lst = by_sum[s]
        for a in range(len(lst)):
            for c in range(a + 1, len(lst)):
                p, q = lst[a], lst[c]
                if set(p) & set(q):
                    continue
                exch.append((p, q))
    return comb, exch


def _cycle_draw(rng: np.random.Generator, cands: list, n: int) -> list:
    """n draws by cycling through one seeded shuffle of the distinct candidates.

    Duplicated equations (independent Arrhenius draws) appear only once every distinct
    candidate has been used.
    """
    if n == 0:
        return []
    order = rng.permutation(len(cands))
    return [cands[order[k % len(cands)]] for k in range(n)]


def _nasa7_from_cp_poly(cp_coeffs_T: np.ndarray, hf_R: float, s_R: float) -> np.ndarray:
    """Seven NASA coefficients for a cp/R cubic in T, fixed by h(T_REF) and s(T_REF).

    ``cp_coeffs_T`` holds a1..a4 of cp/R = a1 + a2 T + a3 T^2 + a4 T^3 (a5 = 0).
    a6 is chosen so that h/R at T_REF equals ``hf_R`` and a7 so that s/R at T_REF
    equals ``s_R`` (standard NASA-7 integration constants).
    """
    a1, a2, a3, a4 = (float(v) for v in cp_coeffs_T)
    a5 = 0.0
    T = T_REF
    a6 = hf_R - (a1 * T + a2 * T ** 2 / 2 + a3 * T ** 3 / 3 + a4 * T ** 4 / 4)
    a7 = s_R - (a1 * math.log(T) + a2 * T + a3 * T ** 2 / 2 + a4 * T ** 3 / 3)
    return np.array([a1, a2, a3, a4, a5, a6, a7], dtype=np.float64)


def _smoothstep_cp_coeffs(c_lo: float, c_hi: float) -> np.ndarray:
    """cp/R = c_lo + (c_hi - c_lo) S(x), S = 3x^2 - 2x^3, x = (T - 300)/4700, as a cubic in T."""
    p = 1.0 / (T_FIT_HI - T_FIT_LO)
    q = -T_FIT_LO / (T_FIT_HI - T_FIT_LO)
    x = np.polynomial.Polynomial([q, p])
    S = 3.0 * x ** 2 - 2.0 * x ** 3
    cp = c_lo + (c_hi - c_lo) * S
    c = np.zeros(4)
    c[: len(cp.coef)] = cp.coef
    return c


def make_mechanism(recipe: MechRecipe) -> Mechanism:
    """Build the synthetic mechanism of a recipe (deterministic in ``recipe.seed``)."""
    rng = np.random.default_rng(recipe.seed)
    E, ns, R = recipe.n_elements, recipe.n_species, recipe.n_reactions
    n_tb = _round_half_up(recipe.frac_third_body * R)
    n_irr = _round_half_up(recipe.frac_irreversible * R)
    n_ex = R - n_tb
    all_comps = np.array([c for c in itertools.product(range(3), repeat=E) if any(c)], dtype=np.int8)

    for _attempt in range(10000):
        sel = rng.choice(len(all_comps), ns, replace=False)
        comps = all_comps[sel]
        comb, exch = _candidates(comps)
        if len(comb) < max(n_tb, 1 if n_tb else 0) or len(exch) < (1 if n_ex else 0):
            continue
        comb_draw = _cycle_draw(rng, comb, n_tb)
        exch_draw = _cycle_draw(rng, exch, n_ex)
        covered = set()
        for (i, j, k) in comb_draw:
            covered |= {i, j, k}
        for (p, q) in exch_draw:
            covered |= set(p) | set(q)
        if len(covered) == ns:
            break
    else:  # pragma: no cover - recipes in this module always succeed quickly
        raise RuntimeError(f"no composition set covers every species for {recipe.name}")

    # Species thermodynamics, drawn before the reactions are oriented.  Formation enthalpy:
    # hf/R = -hf_bond_R (n_atoms - 1) + U[-w, w], i.e. every bond formed releases about
    # hf_bond_R, so a combination A + B -> C is exothermic by hf_bond_R +- 3w.  Standard
    # entropy s/R = 20 + 2 n_atoms + U[-2, 2].  cp/R: smooth step from c_lo to c_hi.
    lo_c, hi_c = recipe.cp_range
    w = recipe.hf_noise_R
    thermo_draws = []
    for s in range(ns):
        c_lo = rng.uniform(lo_c, 5.0)
        c_hi = rng.uniform(c_lo, hi_c)
        n_atoms = int(comps[s].sum())
        hf_R = -recipe.hf_bond_R * (n_atoms - 1) + rng.uniform(-w, w)
        s_R = 20.0 + 2.0 * n_atoms + rng.uniform(-2.0, 2.0)
        thermo_draws.append((c_lo, c_hi, hf_R, s_R))
    hf = np.array([t[2] for t in thermo_draws])

    # Reaction list.  Exchange entries are written in their exothermic direction (standard
    # reaction enthalpy <= 0 at 298.15 K), so that the reverse rate obtained through the
    # equilibrium constant is the slower one; combinations read A + B (+M) <=> C.
    rxns = []
    for (p, q) in exch_draw:
        if recipe.exothermic_forward:
            if hf[list(q)].sum() > hf[list(p)].sum():
                p, q = q, p
        elif rng.random() < 0.5:
            p, q = q, p
        rxns.append(("ex", p, q))
    for (i, j, k) in comb_draw:
        rxns.append(("tb", (i, j), (k,)))
    order = rng.permutation(len(rxns))
    rxns = [rxns[o] for o in order]

    def pack(species: Sequence[int]):
        idx = [-1] * MAX_SLOTS
        nu = [0] * MAX_SLOTS
        uniq = []
        for s in species:
            if s in uniq:
                nu[uniq.index(s)] += 1
            else:
                uniq.append(s)
                idx[len(uniq) - 1] = s
                nu[len(uniq) - 1] = 1
        return idx, nu

    reac_idx = np.full((R, MAX_SLOTS), -1, np.int32)
    reac_nu = np.zeros((R, MAX_SLOTS), np.int32)
    prod_idx = np.full((R, MAX_SLOTS), -1, np.int32)
    prod_nu = np.zeros((R, MAX_SLOTS), np.int32)
    tb = np.full(R, -1, np.int32)
    k_tb = 0
    for r, (kind, lhs, rhs) in enumerate(rxns):
        reac_idx[r], reac_nu[r] = pack(lhs)
        prod_idx[r], prod_nu[r] = pack(rhs)
        if kind == "tb":
            tb[r] = k_tb
            k_tb += 1

    reversible = np.ones(R, np.int32)
    if n_irr:
        reversible[rng.choice(R, n_irr, replace=False)] = 0

    A = 10.0 ** rng.uniform(*recipe.logA_range, size=R)
    b = rng.uniform(*recipe.b_range, size=R)
    Ta = rng.uniform(*recipe.Ta_range, size=R)
    eff = rng.uniform(*recipe.eff_range, size=(n_tb, ns))

    elements = ELEMENT_ORDER[:E]
    masses = np.array([ELEMENT_MASS[e] for e in elements])
    M = comps.astype(np.float64) @ masses

    nasa = np.zeros((ns, 2, 7))
    for s, (c_lo, c_hi, hf_R, s_R) in enumerate(thermo_draws):
        coef = _nasa7_from_cp_poly(_smoothstep_cp_coeffs(c_lo, c_hi), hf_R, s_R)
        nasa[s, 0] = coef
        nasa[s, 1] = coef

    return Mechanism(
        name=recipe.name, elements=tuple(elements), comp=comps.astype(np.int8), M=M, nasa=nasa,
        T_lo=np.full(ns, T_FIT_LO), T_mid=np.full(ns, T_FIT_MID), T_hi=np.full(ns, T_FIT_HI),
        reac_idx=reac_idx, reac_nu=reac_nu, prod_idx=prod_idx, prod_nu=prod_nu,
        A=A, b=b, Ta=Ta, reversible=reversible, tb=tb, eff=eff)


_MECH_CACHE: Dict[str, Mechanism] = {}


def mechanism(name: str) -> Mechanism:
    """The named synthetic mechanism ("mech9" or "mech36"), built once per process."""
    if name not in _MECH_CACHE:
        _MECH_CACHE[name] = make_mechanism(RECIPES[name])
    return _MECH_CACHE[name]


def mechanism_from_lists(name: str, elements: Sequence[str], comp, nasa, reactions,
                         eff=None, T_mid=None) -> Mechanism:
    """Assemble a small hand-written mechanism (test fixtures).

    ``reactions``: list of dicts with keys ``reac`` and ``prod`` (lists of (species, nu)),
    ``A``, ``b``, ``Ta``, optional ``reversible`` (default True) and ``tb`` (row of ``eff``
    or -1).
    """
    comp = np.asarray(comp, np.int8)
    ns = comp.shape[0]
    masses = np.array([ELEMENT_MASS[e] for e in elements])
    nasa = np.asarray(nasa, np.float64).reshape(ns, 2, 7)
    R = len(reactions)
    reac_idx = np.full((R, MAX_SLOTS), -1, np.int32)
    reac_nu = np.zeros((R, MAX_SLOTS), np.int32)
    prod_idx = np.full((R, MAX_SLOTS), -1, np.int32)
    prod_nu = np.zeros((R, MAX_SLOTS), np.int32)
    A = np.zeros(R); b = np.zeros(R); Ta = np.zeros(R)
    rev = np.ones(R, np.int32); tb = np.full(R, -1, np.int32)
    for r, rx in enumerate(reactions):
        for k, (s, n) in enumerate(rx["reac"]):
            reac_idx[r, k], reac_nu[r, k] = s, n
        for k, (s, n) in enumerate(rx["prod"]):
            prod_idx[r, k], prod_nu[r, k] = s, n
        A[r], b[r], Ta[r] = rx["A"], rx.get("b", 0.0), rx.get("Ta", 0.0)
        rev[r] = 1 if rx.get("reversible", True) else 0
        tb[r] = rx.get("tb", -1)
    eff = np.zeros((0, ns)) if eff is None else np.asarray(eff, np.float64).reshape(-1, ns)
    T_mid = np.full(ns, T_FIT_MID) if T_mid is None else np.asarray(T_mid, np.float64)
    return Mechanism(name=name, elements=tuple(elements), comp=comp, M=comp.astype(np.float64) @ masses,
                     nasa=nasa, T_lo=np.full(ns, T_FIT_LO), T_mid=T_mid, T_hi=np.full(ns, T_FIT_HI),
                     reac_idx=reac_idx, reac_nu=reac_nu, prod_idx=prod_idx, prod_nu=prod_nu,
                     A=A, b=b, Ta=Ta, reversible=rev, tb=tb, eff=eff)


# ----------------------------------------------------------------------------------------------
# Cell states.  Layout: rho[n], T[n], Y[Ns][n] (species-major, cell index fastest).
# ----------------------------------------------------------------------------------------------

@dataclasses.dataclass
class CellStates:
    rho: np.ndarray   # [n] kg/m^3
    T: np.ndarray     # [n] K
    Y: np.ndarray     # [Ns][n] mass fractions

    @property
    def n(self) -> int:
        return int(self.rho.shape[0])

    def subset(self, idx) -> "CellStates":
        idx = np.asarray(idx)
        return CellStates(np.ascontiguousarray(self.rho[idx]), np.ascontiguousarray(self.T[idx]),
                          np.ascontiguousarray(self.Y[:, idx]))


def uniform_cells(seed: int, n: int, ns: int, alpha: float,
                  T_range=(1000.0, 3000.0), rho_range=(0.01, 1.0)) -> CellStates:
    """rho log-uniform, T uniform, Y ~ Dirichlet(alpha * ones(ns))."""
    rng = np.random.default_rng(seed)
    rho = 10.0 ** rng.uniform(math.log10(rho_range[0]), math.log10(rho_range[1]), size=n)
    T = rng.uniform(T_range[0], T_range[1], size=n)
    Y = rng.dirichlet(np.full(ns, alpha), size=n).T
    return CellStates(np.ascontiguousarray(rho), np.ascontiguousarray(T), np.ascontiguousarray(Y))


def band_grid_cells(seed: int, ns: int, nx: int = 1024, ny: int = 1024) -> CellStates:
    """Shock-heated band on an nx x ny grid over [0,1)^2 (cell index = j*nx + i).

    B = exp(-((x - x_c(y))/0.08)^2), x_c = 0.5 + 0.05 sin(2 pi y);
    T = 800 + 2400 B + N(0, 25 K) clamped to [800, 3200];
    rho = 0.05 * 20^B * (1 + U[-0.05, 0.05]) clamped to [0.05, 1]; Y ~ Dirichlet(1).
    """
    rng = np.random.default_rng(seed)
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    X, Yg = np.meshgrid(x, y)  # [ny][nx]
    xc = 0.5 + 0.05 * np.sin(2.0 * np.pi * Yg)
    B = np.exp(-(((X - xc) / 0.08) ** 2)).ravel()
    n = nx * ny
    T = np.clip(800.0 + 2400.0 * B + rng.normal(0.0, 25.0, size=n), 800.0, 3200.0)
    rho = np.clip(0.05 * 20.0 ** B * (1.0 + rng.uniform(-0.05, 0.05, size=n)), 0.05, 1.0)
    Y = rng.dirichlet(np.ones(ns), size=n).T
    return CellStates(np.ascontiguousarray(rho), np.ascontiguousarray(T), np.ascontiguousarray(Y))


# Workloads ------------------------------------------------------------------------------------

DT_DEFAULT = 1.0e-6


def workload_small_mech9(n: int = 4096) -> Tuple[Mechanism, CellStates, float]:
    """9-species/38-reaction mechanism, 4096 cells, one step of 1e-6 s (seed 0)."""
    m = mechanism("mech9")
    return m, uniform_cells(0, n, m.ns, 1.0), DT_DEFAULT


def workload_grid_mech9(nx: int = 1024, ny: int = 1024) -> Tuple[Mechanism, CellStates, float]:
    """9-species/38-reaction mechanism on a 1024x1024 band grid (seed 1), steps of 1e-6 s."""
    m = mechanism("mech9")
    return m, band_grid_cells(1, m.ns, nx, ny), DT_DEFAULT


def workload_mech36(n: int = 1 << 18) -> Tuple[Mechanism, CellStates, float]:
    """36-species/308-reaction mechanism, 2^18 cells, Dirichlet(0.5) (seed 2), dt 1e-6 s."""
    m = mechanism("mech36")
    return m, uniform_cells(2, n, m.ns, 0.5), DT_DEFAULT


@dataclasses.dataclass
class Instance:
    mech: str
    n_cells: int
    dt: float
    state_seed: int

    def states(self) -> CellStates:
        m = mechanism(self.mech)
        alpha = 1.0 if self.mech == "mech9" else 0.5
        return uniform_cells(self.state_seed, self.n_cells, m.ns, alpha)


def batch_instances(seed: int = 3, n_inst: int = 64, min_cells: int = 1024, max_cells: int = 262144,
                    dt_range=(1.0e-7, 1.0e-5)) -> List[Instance]:
    """Uneven batch: each instance mech9 or mech36 with probability 1/2, cells log-uniform, dt uniform."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_inst):
        mech = "mech9" if rng.random() < 0.5 else "mech36"
        n = int(round(math.exp(rng.uniform(math.log(min_cells), math.log(max_cells)))))
        dt = float(rng.uniform(*dt_range))
        out.append(Instance(mech, n, dt, state_seed=1000 * seed + k))
    return out


@dataclasses.dataclass
class Request:
    arrival: float  # s after the start of the run
    inst: Instance


def serving_requests(seed: int, n_req: int, rate_per_s: float, frac_mech9: float = 0.7,
                     median_cells: int = 16384, sigma_ln: float = 1.0,
                     cells_range=(1024, 524288), dt_range=(1.0e-7, 1.0e-5)) -> List[Request]:
    """Poisson arrivals; log-normal request sizes; 70/30 mech9/mech36 mix; dt uniform."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n_req):
        t += rng.exponential(1.0 / rate_per_s)
        mech = "mech9" if rng.random() < frac_mech9 else "mech36"
        n = int(np.clip(round(math.exp(rng.normal(math.log(median_cells), sigma_ln))), *cells_range))
        dt = float(rng.uniform(*dt_range))
        out.append(Request(t, Instance(mech, n, dt, state_seed=100000 * seed + k)))
    return out


def mean_request_cells(median_cells: int = 16384, sigma_ln: float = 1.0) -> float:
    """Mean of the (unclamped) log-normal request size."""
    return median_cells * math.exp(0.5 * sigma_ln ** 2)
