"""The C-ABI library loads, exports every function include/kin.h declares, and generates and
compiles a mechanism's lane-layout kernels for gfx950 (hipRTC needs no device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "kin.h")).read()
    return sorted(set(re.findall(r"^\s*(?:kin_status|void|const char \*)\s*(kin_\w+)\s*\(", src, re.M)))


def test_library_exports_header():
    from paper_1110_4903_amd import kin
    lib = ctypes.CDLL(kin.SO)
    names = declared_functions()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(kin.EXPORTS)


def test_default_solver_opts_match_oracle_defaults(orc):
    """Both sides document the same default Newton controls (numbers, not shared code)."""
    from paper_1110_4903_amd import kin
    s = kin.solver_opts()
    o = orc.default_opts()
    for f in ("rtol", "atol_Y", "atol_T", "y_neg", "k_max", "L_max", "max_iters", "point_implicit", "diverge_ratio"):
        assert getattr(s, f) == getattr(o, f), f
    assert s.L_forced == -1 and s.layout == kin.LAYOUT_AUTO


def test_jit_compiles_mech9():
    from paper_1110_4903_amd import kin, synth
    log = kin.jit_check(synth.mechanism("mech9"))
    assert log.startswith("compiled")


def test_mechanism_validation():
    from paper_1110_4903_amd import kin, synth
    m = synth.mechanism("mech9")
    bad = synth.Mechanism(**{**m.__dict__})
    bad.reac_idx = m.reac_idx.copy()
    bad.reac_idx[0, 0] = 99
    with pytest.raises(kin.KinError) as e:
        kin.jit_check(bad)
    assert e.value.status == kin.EINVAL
    bad = synth.Mechanism(**{**m.__dict__})
    bad.prod_nu = m.prod_nu.copy()
    bad.prod_nu[0, 0] = 2   # breaks the element balance
    with pytest.raises(kin.KinError):
        kin.jit_check(bad)
    with pytest.raises(kin.KinError):
        kin.jit_check(synth.mechanism("mech36"))  # 36 species exceed the lane layout


def test_c_program_compiles_against_header(tmp_path):
    """The plain-C check program (tests/abi_c/kin_abi_check.c) compiles and links against
    include/kin.h and libkin.so with a C compiler alone (its GPU run is a separate test)."""
    import shutil
    import subprocess
    from paper_1110_4903_amd import kin
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    exe = tmp_path / "kin_abi_check"
    src = os.path.join(ROOT, "tests", "abi_c", "kin_abi_check.c")
    libdir = os.path.dirname(kin.SO)
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"), src,
                        "-L", libdir, "-lkin", "-lm", "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


# Sections of the paper (Le & Cambier, arXiv:1110.4903): 1 Introduction, 2 Governing
# Equations, 3 Numerical Formulation (3.1 Fluid Dynamics, 3.2 Chemical Kinetics), 4 GPU
# Implementation (4.1 Computational Fluid Dynamics, 4.2 Chemical Kinetics), 5 Results (5.1 Solver
# Results, 5.2 Performance Results), 6 Conclusion, Appendix A.
PAPER_SECTIONS = {"1", "2", "3", "3.1", "3.2", "4", "4.1", "4.2", "5", "5.1", "5.2", "6"}
# Calls that serve no passage of the paper (library plumbing) say so explicitly.
PLUMBING = {"kin_last_error", "kin_destroy", "kin_sync", "kin_fluid_release"}
# The allocation-free advance names the callers it is for in place of a passage.
NO_ALLOC = {"kin_advance_noalloc"}


def export_comments():
    """The comment block directly above each declared export (its contract)."""
    src = open(os.path.join(ROOT, "include", "kin.h")).read()
    out = {}
    for m in re.finditer(r"/\*((?:(?!\*/).)*)\*/\s*(?:kin_status|void|const char \*)\s*(kin_\w+)\s*\(", src, re.S):
        out[m.group(2)] = m.group(1)
    return out


def test_every_export_cites_the_paper():
    """Each exported call's comment has a 'Paper:' line; every call that is not plumbing names
    at least one section, and every section cited anywhere in the header exists in the paper."""
    comments = export_comments()
    names = declared_functions()
    assert set(comments) == set(names), set(names) ^ set(comments)
    src = open(os.path.join(ROOT, "include", "kin.h")).read()
    for sec in re.findall(r"Sec\. (\d+(?:\.\d+)?)", src):
        assert sec in PAPER_SECTIONS, sec
    for n, c in comments.items():
        assert "Paper:" in c, n
        cite = c[c.index("Paper:"):]
        if n in PLUMBING:
            assert "no passage" in cite, n
        elif n in NO_ALLOC:
            assert "cannot allocate" in cite, n
        else:
            assert re.search(r"Sec\. \d", cite), n
