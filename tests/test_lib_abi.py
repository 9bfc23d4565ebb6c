"""The C-ABI library loads and exports every symbol the header declares;
host-side argument checks (no GPU needed: no compute is launched)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgseg.h")


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (load torch's HIP runtime first, as the binding does)
    from paper_1807_02137_amd import build, mgseg
    if not os.path.exists(build.LIB):
        build.build()
    return mgseg.lib()


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mgseg_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_params_struct_matches(lib):
    from paper_1807_02137_amd import mgseg
    p = mgseg._Params()
    lib.mgseg_params_default(C.byref(p))
    assert p.struct_size == C.sizeof(mgseg._Params)
    d = mgseg.Params()
    for f in ("mu", "lambda1", "theta", "M", "Sigma", "eps_tv_px", "nu1", "nu2", "coarse_iters", "smoother"):
        assert getattr(p, f) == getattr(d, f), f


def test_strerror(lib):
    for code in range(8):
        assert lib.mgseg_strerror(code)


def test_setup_rejects_bad_arguments_before_any_device_work(lib):
    from paper_1807_02137_amd import mgseg
    p = mgseg.Params().to_c()
    mk = (C.c_float * 6)(10, 10, 10, 20, 20, 15)
    out = C.c_void_p()
    img = C.c_void_p(16)  # never dereferenced: the checks below fail first
    # null image
    assert lib.mgseg_setup(None, 64, 64, 64, mk, 3, C.byref(p), None, C.byref(out)) == 1
    # pitch < m
    assert lib.mgseg_setup(img, 64, 64, 32, mk, 3, C.byref(p), None, C.byref(out)) == 1
    # no markers
    assert lib.mgseg_setup(img, 64, 64, 64, mk, 0, C.byref(p), None, C.byref(out)) == 1
    # bad struct size
    q = mgseg.Params().to_c(); q.struct_size = 4
    assert lib.mgseg_setup(img, 64, 64, 64, mk, 3, C.byref(q), None, C.byref(out)) == 1
    # shape not divisible by 2^(levels-1)
    r = mgseg.Params(levels=4).to_c()
    assert lib.mgseg_setup(img, 60, 64, 64, mk, 3, C.byref(r), None, C.byref(out)) == 2
    # non-finite marker
    bad = (C.c_float * 6)(10, float("nan"), 10, 20, 20, 15)
    assert lib.mgseg_setup(img, 64, 64, 64, bad, 3, C.byref(p), None, C.byref(out)) == 1
    # marker outside the image
    far = (C.c_float * 6)(10, 10, 64, 20, 20, 15)
    assert lib.mgseg_setup(img, 64, 64, 64, far, 3, C.byref(p), None, C.byref(out)) == 1
    neg = (C.c_float * 6)(10, 10, 10, -0.5, 20, 15)
    assert lib.mgseg_setup(img, 64, 64, 64, neg, 3, C.byref(p), None, C.byref(out)) == 1
    # a grid of one row or column
    assert lib.mgseg_setup(img, 1, 64, 64, mk, 3, C.byref(mgseg.Params(levels=1).to_c()), None, C.byref(out)) == 1
    # Rada-Chen needs a marker polygon of positive area: at least 3 markers
    rc = mgseg.Params(model=1).to_c()
    assert lib.mgseg_setup(img, 64, 64, 64, mk, 2, C.byref(rc), None, C.byref(out)) == 1
    # the column-system smoothers (Hybrid Smoother 1, GSLINE-I, GSLINE-II) take one workgroup per
    # column: columns of more than 1024 cells are refused (rows may be longer)
    for sm in (2, 3, 6):
        q = mgseg.Params(smoother=sm, levels=3).to_c()
        assert lib.mgseg_setup(img, 2048, 64, 64, mk, 3, C.byref(q), None, C.byref(out)) == 1
    assert not out.value
    # network sizes
    net = C.c_void_p()
    for base, depth in ((8, 3), (24, 3), (0, 3), (16, 1), (16, 7), (64, 5)):
        assert lib.mgseg_net_create(base, depth, 0, C.byref(net)) == 1
    assert not net.value
    # checkpoint and batch entry points with null handles
    n = C.c_size_t(0)
    assert lib.mgseg_get_state(None, None, C.byref(n)) == 1
    assert lib.mgseg_set_state(None, None, 0) == 1
    assert lib.mgseg_solve_batch(None, 1e-6, 10, None, None) == 1
    # the network's Adam state with a null handle
    steps = C.c_longlong(0)
    assert lib.mgseg_net_get_adam(None, None, None, C.byref(steps)) == 1
    assert lib.mgseg_net_set_adam(None, None, None, C.c_longlong(0)) == 1
    # null context everywhere
    assert lib.mgseg_vcycle(None, None) == 1
    assert lib.mgseg_solve(None, 1e-6, 10, None, None) == 1
    lib.mgseg_destroy(None)
