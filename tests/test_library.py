"""Host-side checks of the C-ABI library (no GPU needed): it loads and
exports every symbol include/mfdkc.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "mfdkc.h")
LIB = os.path.join(ROOT, "paper_2503_19379_amd", "libmfdkc.so")


def declared():
    txt = open(HDR).read()
    return sorted(set(re.findall(r"\b(mfd_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = declared()
    for n in ["mfd_build", "mfd_op_apply", "mfd_precond_solve", "mfd_bands", "mfd_destroy", "mfd_lambda_re"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_only_calls():
    from paper_2503_19379_amd import binding as b
    L = b.lib()
    assert L.mfd_strerror(-1) == b"invalid argument"
    assert b.mfd_supported_n(64) and b.mfd_supported_n(24) and b.mfd_supported_n(96) and b.mfd_supported_n(150)
    assert not b.mfd_supported_n(7) and not b.mfd_supported_n(2)
    o = b.default_opts()
    assert o.max_iter > 0 and o.max_gamma_doublings == 4
    assert b.max_block() >= 21
    # argument validation happens before any device work
    h = ctypes.c_void_p()
    assert L.mfd_build(8, 1.0, 2, None, None, ctypes.byref(h)) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_side_argument_errors():
    """Argument checks that return before any device call."""
    from paper_2503_19379_amd import binding as b
    L = b.lib()
    h = ctypes.c_void_p()
    assert L.mfd_mlp_create(0, 8, 1, 4, 2, 1, 0, ctypes.byref(h)) == -1
    assert L.mfd_mlp_create(8, 0, 1, 4, 2, 1, 0, ctypes.byref(h)) == -1
    assert L.mfd_mlp_create(8, 8, 1, 4, 0, 1, 0, ctypes.byref(h)) == -1
    assert L.mfd_tuning(None, None) == -1
    assert L.mfd_set_tuning(None, None) == -1
    eps = (ctypes.c_double * 512)(*([1.0] * 512))
    dp = ctypes.cast(eps, ctypes.POINTER(ctypes.c_double))
    assert L.mfd_build(8, 1.0, 3, dp, None, ctypes.byref(h)) == -6      # order 3: unsupported
    assert L.mfd_build(8, 1.0, 10, dp, None, ctypes.byref(h)) == -6
    assert L.mfd_build(7, 1.0, 2, dp, None, ctypes.byref(h)) == -6      # no FFT plan for N = 7
    eps[5] = -1.0
    assert L.mfd_build(8, 1.0, 2, dp, None, ctypes.byref(h)) == -1      # eps must be > 0
    mu = (ctypes.c_double * 1536)(*([1.0] * 1536))                       # 3 N^3 edges at N = 8
    mp = ctypes.cast(mu, ctypes.POINTER(ctypes.c_double))
    assert L.mfd_build_mu(8, 1.0, 2, None, None, ctypes.byref(h)) == -1  # NULL mu
    assert L.mfd_build_mu(7, 1.0, 2, mp, None, ctypes.byref(h)) == -6    # no FFT plan for N = 7
    assert L.mfd_build_mu(8, 0.0, 2, mp, None, ctypes.byref(h)) == -1    # L must be > 0
    mu[1500] = 0.0                                                       # an e_3 entry
    assert L.mfd_build_mu(8, 1.0, 2, mp, None, ctypes.byref(h)) == -1    # mu must be > 0
    mu[1500] = float("nan")
    assert L.mfd_build_mu(8, 1.0, 2, mp, None, ctypes.byref(h)) == -1
    # general lattice: NULL, singular and non-finite lattice matrices
    eps = (ctypes.c_double * 512)(*([1.0] * 512))
    ep = ctypes.cast(eps, ctypes.POINTER(ctypes.c_double))
    bcc = (ctypes.c_double * 9)(-0.5, 0.5, 0.5, 0.5, -0.5, 0.5, 0.5, 0.5, -0.5)
    lp = ctypes.cast(bcc, ctypes.POINTER(ctypes.c_double))
    assert L.mfd_build_lattice(8, None, 2, ep, None, ctypes.byref(h)) == -1
    assert L.mfd_build_lattice(8, lp, 2, None, None, ctypes.byref(h)) == -1
    assert L.mfd_build_lattice(7, lp, 2, ep, None, ctypes.byref(h)) == -6
    assert L.mfd_build_lattice(8, lp, 3, ep, None, ctypes.byref(h)) == -6
    sing = (ctypes.c_double * 9)(1.0, 2.0, 0.0, 2.0, 4.0, 0.0, 3.0, 6.0, 1.0)   # a_2 = 2 a_1
    assert L.mfd_build_lattice(8, ctypes.cast(sing, ctypes.POINTER(ctypes.c_double)), 2, ep, None,
                               ctypes.byref(h)) == -1
    bcc[4] = float("inf")
    assert L.mfd_build_lattice(8, lp, 2, ep, None, ctypes.byref(h)) == -1
    assert h.value is None
    o = b.default_opts()
    assert o.autotune == 1 and o.stall_window == 40 and o.learn_steps == 30
    assert o.cold_start == 0 and o.balance == 0 and o.hard_lock == 0


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of mfd_opts and mfd_kstats have the C layout: every
    field's offset and the struct sizes, from a C program compiled against
    include/mfdkc.h."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    from paper_2503_19379_amd import binding as B
    lines = []
    for st in (B.mfd_opts, B.mfd_kstats):
        cname = st.__name__
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "mfdkc.h"\nint main(void) {\n    '
                   + "\n    ".join(lines) + "\n    return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for st in (B.mfd_opts, B.mfd_kstats):
        cname = st.__name__
        assert got[(cname, "sizeof")] == ctypes.sizeof(st), cname
        for f, _ in st._fields_:
            assert got[(cname, f)] == getattr(st, f).offset, (cname, f)
