"""The C-ABI library loads and exports every symbol that include/ertvie.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "ertvie.h")) as fh:
        src = fh.read()
    return sorted(set(re.findall(r"ERT_API\s+[\w\s\*]+?\b(ert_vie_\w+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("ert_vie_plan", "ert_vie_apply", "ert_vie_solve", "ert_vie_destroy", "ert_vie_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1610_00835_amd import ertvie
    L = ertvie.load()
    for name in _declared():
        assert hasattr(L, name), name
        assert isinstance(getattr(L, name), ctypes._CFuncPtr)


def test_strerror_and_null_plan_without_gpu():
    from paper_1610_00835_amd import ertvie
    L = ertvie.load()
    assert ertvie.strerror(0) == "ok"
    assert "invalid" in ertvie.strerror(-1)
    assert L.ert_vie_size(None) == -1
    L.ert_vie_destroy(None)
    # argument validation returns before any device work
    assert L.ert_vie_apply(None, 1, None, None, 1) == ertvie.EINVAL
    assert L.ert_vie_solve(None, None, None, 1, None, None) == ertvie.EINVAL


def test_plan_rejects_bad_arguments_before_device_use():
    import numpy as np
    from paper_1610_00835_amd import ertvie
    L = ertvie.load()
    N = 16
    st = np.full(N, 2.0)
    ss = np.full(N, 1.0)
    dp = ctypes.POINTER(ctypes.c_double)

    def plan(**kw):
        o = ertvie.VieOpts()
        o.dim, o.h, o.kernel, o.method, o.prec = 2, 0.25, 0, 0, 0
        o.n[0], o.n[1], o.n[2] = 4, 4, 1
        sig_t = kw.pop("st", st)
        sig_s = kw.pop("ss", ss)
        for k, v in kw.items():
            setattr(o, k, v)
        h = ctypes.c_void_p()
        return L.ert_vie_plan(ctypes.byref(o), np.ascontiguousarray(sig_t).ctypes.data_as(dp),
                              np.ascontiguousarray(sig_s).ctypes.data_as(dp), None, ctypes.byref(h))
    assert plan(dim=4) == ertvie.EINVAL
    assert plan(h=0.0) == ertvie.EINVAL
    assert plan(h=float("nan")) == ertvie.EINVAL
    assert plan(flags=1) == ertvie.EINVAL
    assert plan(cheb_n=12) == ertvie.EINVAL
    assert plan(st=np.where(np.arange(N) == 3, -1.0, 2.0)) == ertvie.EINVAL
    assert plan(ss=np.full(N, 2.5)) == ertvie.EINVAL           # absorption < 0
    assert plan(ss=np.full(N, -0.1)) == ertvie.EINVAL
    assert plan(st=np.linspace(1, 2, N)) == ertvie.EINVAL      # homogeneous kernel needs constant sigma_t
