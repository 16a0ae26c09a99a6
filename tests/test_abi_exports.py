"""The C-ABI library loads and exports every symbol that include/ertvie.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "ertvie.h")) as fh:
        src = fh.read()
    return sorted(set(re.findall(r"ERT_API\s+[\w\s\*]+?\b(ert_(?:vie|net)_\w+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("ert_vie_plan", "ert_vie_apply", "ert_vie_solve", "ert_vie_destroy", "ert_vie_strerror",
                 "ert_vie_fft_precond", "ert_vie_fft_info", "ert_vie_transport", "ert_vie_diff_precond", "ert_net_create", "ert_net_forward", "ert_net_grad", "ert_net_train_step", "ert_net_destroy"):
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
    assert L.ert_vie_fft_precond(None, None, None, 1) == ertvie.EINVAL
    assert L.ert_vie_fft_info(None, None) == ertvie.EINVAL
    assert L.ert_vie_transport(None, None, None, None, 1, None) == ertvie.EINVAL
    assert L.ert_vie_transport_noalloc(None, None, None, None, 1, None) == ertvie.EINVAL
    assert L.ert_vie_restrict(None, 2, None, None, 1) == ertvie.EINVAL
    assert L.ert_vie_net_apply(None, None, None, None) == ertvie.EINVAL
    assert L.ert_vie_diff_precond(None, None, None, 1) == ertvie.EINVAL
    ms = ctypes.c_double(0.0)
    assert L.ert_vie_read_rate(None, 1 << 20, 4096, 3, None, ctypes.byref(ms)) == ertvie.EINVAL
    assert L.ert_vie_read_rate(ctypes.c_void_p(4096), 1 << 20, 4008, 3, None, ctypes.byref(ms)) == ertvie.EINVAL


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
            if k == "form":
                o.form[0], o.form[1] = v
            else:
                setattr(o, k, v)
        h = ctypes.c_void_p()
        return L.ert_vie_plan(ctypes.byref(o), np.ascontiguousarray(sig_t).ctypes.data_as(dp),
                              np.ascontiguousarray(sig_s).ctypes.data_as(dp), None, ctypes.byref(h))
    assert plan(dim=4) == ertvie.EINVAL
    assert plan(h=0.0) == ertvie.EINVAL
    assert plan(h=float("nan")) == ertvie.EINVAL
    assert plan(scheme=2) == ertvie.EINVAL
    assert plan(cheb_n=12) == ertvie.EINVAL
    assert plan(inner_cheb_n=1) == ertvie.EINVAL
    assert plan(inner_cheb_n=9) == ertvie.EINVAL
    assert plan(inner_near16=2) == ertvie.EINVAL
    assert plan(form=(7, 0)) == ertvie.EINVAL                  # execution forms 0..5, stored as f + 1
    assert plan(form=(0, -1)) == ertvie.EINVAL
    assert plan(far_cache_gb=-1.0) == ertvie.EINVAL            # translation-cache budget >= 0, finite
    assert plan(far_cache_gb=float("nan")) == ertvie.EINVAL
    assert plan(far_cache_gb=float("inf")) == ertvie.EINVAL
    assert plan(st=np.where(np.arange(N) == 3, -1.0, 2.0)) == ertvie.EINVAL
    assert plan(ss=np.full(N, 2.5)) == ertvie.EINVAL           # absorption < 0
    assert plan(ss=np.full(N, -0.1)) == ertvie.EINVAL
    assert plan(st=np.linspace(1, 2, N)) == ertvie.EINVAL      # homogeneous kernel needs constant sigma_t


def test_network_arguments_without_gpu():
    """Parameter counts (the canonical layout) and argument checks of the network ABI."""
    from oracle import unet as U
    from paper_1610_00835_amd import ertvie
    ertvie._load_net()
    assert ertvie.Net.param_count() == U.param_count()
    assert ertvie.Net.param_count((16, 16, 32)) == U.param_count((16, 16, 32))
    L = ertvie.load()
    h = ctypes.c_void_p()

    def create(**kw):
        o = ertvie.NetOpts()
        o.dim = kw.pop("dim", 3)
        n = kw.pop("n", (8, 8, 8))
        for a in range(3):
            o.n[a] = n[a]
        for k, v in kw.items():
            if k == "width":
                for a in range(3):
                    o.width[a] = v[a]
            else:
                setattr(o, k, v)
        return L.ert_net_create(ctypes.byref(o), None, ctypes.byref(h))
    assert create(dim=2) == ertvie.EUNSUPPORTED
    assert create(n=(8, 6, 8)) == ertvie.EINVAL          # not a multiple of 4
    assert create(width=(16, 24, 64)) == ertvie.EINVAL   # not a multiple of 16
    assert L.ert_net_size(None) == -1
    L.ert_net_destroy(None)
    assert L.ert_net_forward(None, None, None, None, None, 1) == ertvie.EINVAL
