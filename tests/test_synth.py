"""Generator checks: the synthetic mechanisms follow their recipes (counts, templates, element
balance, thermodynamic ranges) and the candidate search reproduces the paper's Appendix A
reaction set for the hydrogen-air species."""
import os

import numpy as np
import pytest

from paper_1110_4903_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("name", ["mech9", "mech36"])
def test_counts_and_balance(name):
    m = synth.mechanism(name)
    rec = synth.RECIPES[name]
    assert m.ns == rec.n_species and m.nr == rec.n_reactions
    assert int((m.tb >= 0).sum()) == int(np.floor(rec.frac_third_body * rec.n_reactions + 0.5))
    assert int((m.reversible == 0).sum()) == int(np.floor(rec.frac_irreversible * rec.n_reactions + 0.5))
    assert m.ntb == int((m.tb >= 0).sum())
    for r in range(m.nr):
        lhs = np.zeros(m.ne, int)
        rhs = np.zeros(m.ne, int)
        for j in range(3):
            if m.reac_idx[r, j] >= 0:
                lhs += m.reac_nu[r, j] * m.comp[m.reac_idx[r, j]]
            if m.prod_idx[r, j] >= 0:
                rhs += m.prod_nu[r, j] * m.comp[m.prod_idx[r, j]]
        assert np.array_equal(lhs, rhs), m.equation(r)
        reac = set(m.reac_idx[r][m.reac_idx[r] >= 0])
        prod = set(m.prod_idx[r][m.prod_idx[r] >= 0])
        assert not (reac & prod)
        n_reac = m.reac_nu[r].sum()
        n_prod = m.prod_nu[r].sum()
        if m.tb[r] >= 0:
            assert (n_reac, n_prod) == (2, 1)   # A + B (+M) <=> C
        else:
            assert (n_reac, n_prod) == (2, 2)   # A + B <=> C + D
    used = set(m.reac_idx[m.reac_idx >= 0]) | set(m.prod_idx[m.prod_idx >= 0])
    assert used == set(range(m.ns))
    assert np.all((m.eff >= 0.5) & (m.eff <= 3.0))
    assert np.all((m.A >= 1e8) & (m.A <= 1e14))
    assert np.all((m.b >= -1.5) & (m.b <= 1.5))
    assert np.all((m.Ta >= 0) & (m.Ta <= 3e4))
    # molar masses from the element composition
    masses = np.array([synth.ELEMENT_MASS[e] for e in m.elements])
    assert np.allclose(m.M, m.comp @ masses, rtol=0, atol=1e-12)
    assert len({tuple(c) for c in m.comp}) == m.ns


@pytest.mark.parametrize("name", ["mech9", "mech36"])
def test_determinism_and_roundtrip(name, tmp_path):
    a = synth.make_mechanism(synth.RECIPES[name])
    b = synth.make_mechanism(synth.RECIPES[name])
    p = str(tmp_path / f"{name}.npz")
    a.save(p)
    c = synth.Mechanism.load(p)
    for f in ("comp", "M", "nasa", "reac_idx", "reac_nu", "prod_idx", "prod_nu", "A", "b", "Ta",
              "reversible", "tb", "eff", "T_mid"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
        assert np.array_equal(getattr(a, f), getattr(c, f))
    assert c.name == a.name and c.elements == a.elements


@pytest.mark.parametrize("name", ["mech9", "mech36"])
def test_thermo_ranges_and_orientation(name):
    m = synth.mechanism(name)
    T = np.linspace(300.0, 5000.0, 2001)
    for s in range(m.ns):
        a = m.nasa[s, 0]
        assert np.array_equal(m.nasa[s, 0], m.nasa[s, 1])
        cp = a[0] + a[1] * T + a[2] * T ** 2 + a[3] * T ** 3 + a[4] * T ** 4
        assert cp.min() >= 2.5 - 1e-9 and cp.max() <= 8.0 + 1e-9
    # h/R at 298.15 K from the polynomial: every exchange reaction is written downhill and
    # every combination releases enthalpy.
    T0 = 298.15
    a = m.nasa[:, 0]
    hR = a[:, 0] * T0 + a[:, 1] * T0 ** 2 / 2 + a[:, 2] * T0 ** 3 / 3 + a[:, 3] * T0 ** 4 / 4 + a[:, 5]
    for r in range(m.nr):
        dH = sum(m.prod_nu[r, j] * hR[m.prod_idx[r, j]] for j in range(3) if m.prod_idx[r, j] >= 0) - \
            sum(m.reac_nu[r, j] * hR[m.reac_idx[r, j]] for j in range(3) if m.reac_idx[r, j] >= 0)
        assert dH <= 1e-6, m.equation(r)


def _parse_appendix_a():
    comp = {"H": (1, 0, 0), "O": (0, 1, 0), "H2": (2, 0, 0), "O2": (0, 2, 0), "OH": (1, 1, 0),
            "H2O": (2, 1, 0), "HO2": (1, 2, 0), "H2O2": (2, 2, 0), "N2": (0, 0, 2)}
    eqs = []
    with open(os.path.join(GOLDEN, "appendix_a_h2_air.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            lhs, rhs = line.split("=")
            side = []
            for part in (lhs, rhs):
                sp = []
                for tok in part.split("+"):
                    tok = tok.strip()
                    if tok == "M":
                        continue
                    if tok.startswith("2"):
                        sp += [tok[1:]] * 2
                    else:
                        sp.append(tok)
                side.append(tuple(sorted(sp)))
            eqs.append((side[0], side[1], "M" in line))
    return comp, eqs


def test_candidate_search_reproduces_appendix_a():
    """Appendix A lists 19 reversible H2-air reactions; each one is an element-balanced
    equation of the two templates over the H/O/N compositions, so the generator's candidate
    search over those nine species must contain all of them."""
    comp, eqs = _parse_appendix_a()
    names = list(comp)
    comps = np.array([comp[n] for n in names], np.int8)
    comb, exch = synth._candidates(comps)
    comb_set = {(tuple(sorted((names[i], names[j]))), (names[k],)) for (i, j, k) in comb}
    exch_set = set()
    for (p, q) in exch:
        a = tuple(sorted(names[i] for i in p))
        b = tuple(sorted(names[i] for i in q))
        exch_set |= {(a, b), (b, a)}
    assert len(eqs) == 19
    for lhs, rhs, third in eqs:
        if third:
            two, one = (lhs, rhs) if len(lhs) == 2 else (rhs, lhs)
            assert (two, one) in comb_set, (lhs, rhs)
        else:
            assert (lhs, rhs) in exch_set, (lhs, rhs)
    # the composition set admits 30 distinct template equations in total
    assert len(comb) + len(exch) == 30


def test_states():
    m, st, dt = synth.workload_small_mech9()
    assert st.n == 4096 and dt == 1e-6
    assert np.allclose(st.Y.sum(0), 1.0, atol=1e-12)
    assert st.T.min() >= 1000 and st.T.max() <= 3000
    assert st.rho.min() >= 0.01 and st.rho.max() <= 1.0
    g = synth.band_grid_cells(1, 9, 64, 64)
    assert g.n == 4096 and g.T.min() >= 800 and g.T.max() <= 3200
    assert g.rho.min() >= 0.05 and g.rho.max() <= 1.0
    insts = synth.batch_instances()
    assert len(insts) == 64
    assert all(1024 <= i.n_cells <= 262144 for i in insts)
    assert all(1e-7 <= i.dt <= 1e-5 for i in insts)
    reqs = synth.serving_requests(4, 50, 100.0)
    assert all(reqs[k].arrival < reqs[k + 1].arrival for k in range(49))
    assert all(1024 <= r.inst.n_cells <= 524288 for r in reqs)
