"""Thin ctypes binding of the C ABI in include/ertvie.h (argument marshalling only).

Every step of the computation runs in libertvie.so.  Vectors are torch CUDA
(HIP) float64 tensors: shape (N,) for one right-hand side or (nrhs, N) for
several -- row b of a contiguous (nrhs, N) tensor is column b of the
column-major N x nrhs array the ABI expects.  If the library is missing the
import of this module fails loudly; there is no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libertvie.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
K_HOMOGENEOUS, K_RAY_MIDPOINT = 0, 1
PRECOND_NONE, PRECOND_FFT, PRECOND_DIFFUSION = 0, 1, 2
DIRECT, FMM = 0, 1
FP64, FP32, BF16X3 = 0, 1, 2
OP_G, OP_GS, OP_A = 0, 1, 2

STAGES = ("gather", "near", "p2m", "m2m", "m2l", "l2l", "l2p", "assemble", "direct", "basis", "reduce")
NSTAGES = len(STAGES)

_PREC = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}
_METHOD = {"direct": DIRECT, "fmm": FMM}


class VieOpts(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double),
                ("kernel", ctypes.c_int), ("method", ctypes.c_int), ("prec", ctypes.c_int),
                ("cheb_n", ctypes.c_int), ("leaf", ctypes.c_int), ("nrhs_max", ctypes.c_int),
                ("scheme", ctypes.c_int), ("svd_tol", ctypes.c_double), ("inner_cheb_n", ctypes.c_int),
                ("inner_near16", ctypes.c_int), ("form", ctypes.c_int * 2), ("far_cache_gb", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("restart", ctypes.c_int),
                ("mixed", ctypes.c_int), ("inner_tol", ctypes.c_double), ("rhs_is_phi", ctypes.c_int),
                ("block", ctypes.c_int), ("precond_steps", ctypes.c_int), ("history_max", ctypes.c_int),
                ("precond_kind", ctypes.c_int), ("precond", ctypes.c_void_p), ("history", ctypes.c_void_p)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("matvecs", ctypes.c_int), ("converged", ctypes.c_int),
                ("restarts", ctypes.c_int), ("rel_resid_est", ctypes.c_double),
                ("rel_resid_true", ctypes.c_double), ("t_solve", ctypes.c_double),
                ("rejected", ctypes.c_int), ("precond_applies", ctypes.c_int), ("history_count", ctypes.c_int),
                ("t_setup", ctypes.c_double)]


class NetOpts(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("batch_max", ctypes.c_int),
                ("width", ctypes.c_int * 3), ("reserved", ctypes.c_int * 4)]


class NetTrainOpts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double)]


class FmmInfo(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("leaf", ctypes.c_int), ("cheb_n", ctypes.c_int),
                ("nodes", ctypes.c_int), ("nodes_padded", ctypes.c_int), ("rank", ctypes.c_int * 16),
                ("far_pairs", ctypes.c_long * 16), ("near_pairs", ctypes.c_long), ("form_near", ctypes.c_int),
                ("form_far", ctypes.c_int * 16), ("near_table", ctypes.c_long), ("far_rebuilt", ctypes.c_int * 16),
                ("cache_bytes", ctypes.c_double)]


class FftInfo(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int * 3), ("sigma_t_mean", ctypes.c_double), ("sigma_s_mean", ctypes.c_double),
                ("self_cell", ctypes.c_double), ("symbol_min", ctypes.c_double), ("symbol_max", ctypes.c_double),
                ("bytes", ctypes.c_long)]


class ErtError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        detail = load().ert_vie_last_error().decode()
        super().__init__("%s: %s (status %d)%s" % (where, strerror(status), status,
                                                  (": " + detail) if detail else ""))


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_lib = None


def load():
    """Open libertvie.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libertvie.so is not built (run paper_1610_00835_amd/build.py)")
    # torch ships its own HIP runtime; load it first so that libertvie.so binds to the
    # same libamdhip64 / libhsa-runtime64 (matched by soname) instead of a second copy
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    L.ert_vie_plan.restype = ctypes.c_int
    L.ert_vie_plan.argtypes = [ctypes.POINTER(VieOpts), _dp, _dp, _vp, ctypes.POINTER(_vp)]
    L.ert_vie_apply.restype = ctypes.c_int
    L.ert_vie_apply.argtypes = [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int]
    L.ert_vie_apply_ex.restype = ctypes.c_int
    L.ert_vie_apply_ex.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int]
    L.ert_vie_solve.restype = ctypes.c_int
    L.ert_vie_solve.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.POINTER(SolveOpts),
                                ctypes.POINTER(SolveInfo)]
    L.ert_vie_fft_precond.restype = ctypes.c_int
    L.ert_vie_fft_precond.argtypes = [_vp, _vp, _vp, ctypes.c_int]
    L.ert_vie_transport.restype = ctypes.c_int
    L.ert_vie_transport.argtypes = [_vp, _vp, _vp, _dp, ctypes.c_int, _vp]
    L.ert_vie_net_apply.restype = ctypes.c_int
    L.ert_vie_net_apply.argtypes = [_vp, _vp, _vp, _vp]
    L.ert_vie_restrict.restype = ctypes.c_int
    L.ert_vie_restrict.argtypes = [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int]
    L.ert_vie_read_rate.restype = ctypes.c_int
    L.ert_vie_read_rate.argtypes = [_vp, ctypes.c_size_t, ctypes.c_size_t, ctypes.c_int, _vp,
                                    ctypes.POINTER(ctypes.c_double)]
    L.ert_vie_transport_noalloc.restype = ctypes.c_int
    L.ert_vie_transport_noalloc.argtypes = [_vp, _vp, _vp, _dp, ctypes.c_int, _vp]
    L.ert_vie_diff_precond.restype = ctypes.c_int
    L.ert_vie_diff_precond.argtypes = [_vp, _vp, _vp, ctypes.c_int]
    L.ert_vie_fft_info.restype = ctypes.c_int
    L.ert_vie_fft_info.argtypes = [_vp, ctypes.POINTER(FftInfo)]
    L.ert_vie_diag.restype = ctypes.c_int
    L.ert_vie_diag.argtypes = [_vp, _dp]
    L.ert_vie_size.restype = ctypes.c_long
    L.ert_vie_size.argtypes = [_vp]
    L.ert_vie_destroy.restype = None
    L.ert_vie_destroy.argtypes = [_vp]
    L.ert_vie_profile.restype = ctypes.c_int
    L.ert_vie_profile.argtypes = [_vp, ctypes.c_int, _dp, ctypes.POINTER(ctypes.c_int)]
    L.ert_vie_fmm_info.restype = ctypes.c_int
    L.ert_vie_fmm_info.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(FmmInfo)]
    L.ert_vie_last_error.restype = ctypes.c_char_p
    L.ert_vie_last_error.argtypes = []
    L.ert_vie_strerror.restype = ctypes.c_char_p
    L.ert_vie_strerror.argtypes = [ctypes.c_int]
    _lib = L
    return L


def strerror(status):
    return load().ert_vie_strerror(int(status)).decode()


def read_rate(buf, piece, reps=5, stream=None):
    """Fastest streaming pass over the torch CUDA tensor `buf` in pieces of `piece` bytes per
    workgroup (ert_vie_read_rate): returns (bytes read, milliseconds)."""
    nbytes = buf.numel() * buf.element_size()
    ms = ctypes.c_double(0.0)
    st = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    _check(load().ert_vie_read_rate(ctypes.c_void_p(buf.data_ptr()), nbytes, int(piece), int(reps), st,
                                    ctypes.byref(ms)), "ert_vie_read_rate")
    return nbytes // int(piece) * int(piece), ms.value


def _check(status, where):
    if status != OK:
        raise ErtError(status, where)


def _f64_host(a, N):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if a.size != N:
        raise ValueError("expected %d values, got %d" % (N, a.size))
    return a


def _dev_ptr(t, N, name):
    """Validate a torch CUDA float64 tensor of shape (N,) or (nrhs, N); return (ptr, nrhs)."""
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError("%s must be a float64 CUDA tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.dim() == 1 and t.shape[0] == N:
        return t.data_ptr(), 1
    if t.dim() == 2 and t.shape[1] == N:
        return t.data_ptr(), int(t.shape[0])
    raise ValueError("%s must have shape (N,) or (nrhs, N) with N=%d" % (name, N))


class Plan:
    """An ert_vie plan: the grid, its media and the operator data on the GPU.

    dim, n, h: grid (cell-centred, x fastest); sigma_t, sigma_s: host arrays of N values.
    kernel: 0 homogeneous / 1 midpoint ray rule; method 'direct' | 'fmm';
    prec 'fp64' | 'fp32' | 'bf16x3'.  far_cache_gb: budget of the stored heterogeneous
    translation matrices (0: 90 % of the free device memory); levels over it are rebuilt by
    every apply.
    """

    def __init__(self, dim, n, h, sigma_t, sigma_s, kernel=K_HOMOGENEOUS, method="direct", prec="fp64",
                 cheb_n=0, leaf=0, nrhs_max=1, stream=None, svd_tol=0.0, inner_cheb_n=0, inner_near16=False, scheme=0,
                 form=None, far_cache_gb=0.0):
        L = load()
        n = list(n)[:dim]
        self.dim = int(dim)
        self.n = tuple(int(v) for v in n)
        self.N = int(np.prod(self.n))
        o = VieOpts()
        o.dim = self.dim
        for a in range(3):
            o.n[a] = self.n[a] if a < dim else 1
        o.h = float(h)
        o.kernel = int(kernel)
        o.method = _METHOD[method] if isinstance(method, str) else int(method)
        o.prec = _PREC[prec] if isinstance(prec, str) else int(prec)
        o.cheb_n = int(cheb_n)
        o.leaf = int(leaf)
        o.nrhs_max = int(nrhs_max)
        o.scheme = int(scheme)
        o.svd_tol = float(svd_tol)
        o.inner_cheb_n = int(inner_cheb_n)
        o.inner_near16 = 1 if inner_near16 else 0
        # execution forms of the homogeneous box-offset products: None (timed), f (both
        # products) or (near, far); each 0..5
        if form is not None:
            fn, ff = (form, form) if np.isscalar(form) else form
            o.form[0] = int(fn) + 1
            o.form[1] = int(ff) + 1
        o.far_cache_gb = float(far_cache_gb)
        self.opts = o
        st_h = _f64_host(sigma_t, self.N)
        ss_h = _f64_host(sigma_s, self.N)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        self.stream = stream
        sp = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        handle = _vp()
        _check(L.ert_vie_plan(ctypes.byref(o), st_h.ctypes.data_as(_dp), ss_h.ctypes.data_as(_dp), sp,
                              ctypes.byref(handle)), "ert_vie_plan")
        self._h = handle

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise RuntimeError("plan is closed")
        return self._h

    def apply(self, x, y, op=OP_GS, method=None, prec=None):
        """y = op(x) on the plan's stream (asynchronous)."""
        xp, nx = _dev_ptr(x, self.N, "x")
        yp, ny = _dev_ptr(y, self.N, "y")
        if nx != ny:
            raise ValueError("x and y differ in nrhs")
        if method is None and prec is None:
            st = load().ert_vie_apply(self.handle, int(op), xp, yp, nx)
        else:
            m = self.opts.method if method is None else (_METHOD[method] if isinstance(method, str) else method)
            p = self.opts.prec if prec is None else (_PREC[prec] if isinstance(prec, str) else prec)
            st = load().ert_vie_apply_ex(self.handle, int(op), int(m), int(p), xp, yp, nx)
        _check(st, "ert_vie_apply")
        return y

    def fft_precond(self, r, z):
        """z = M r with the FFT-based preconditioner of the mean medium (asynchronous
        after the first call, which builds it)."""
        rp, nr = _dev_ptr(r, self.N, "r")
        zp, nz = _dev_ptr(z, self.N, "z")
        if nr != nz:
            raise ValueError("r and z differ in nrhs")
        _check(load().ert_vie_fft_precond(self.handle, rp, zp, nr), "ert_vie_fft_precond")
        return z

    def transport(self, U, f, dirs, phi, noalloc=False):
        """Algorithm 1 S.3: phi[k] = Phi(., dirs[k]) for Q = sigma_s U + f (U or f may be None).
        dirs: host (ndir, dim) unit vectors; phi: float64 CUDA tensor (ndir, N).
        noalloc: use ert_vie_transport_noalloc (the library's static device scratch)."""
        dirs = np.ascontiguousarray(dirs, dtype=np.float64)
        if dirs.ndim != 2 or dirs.shape[1] != self.opts.dim:
            raise ValueError("dirs must have shape (ndir, dim)")
        pp, nd = _dev_ptr(phi, self.N, "phi")
        if nd != dirs.shape[0]:
            raise ValueError("phi must have one row per direction")
        up = _dev_ptr(U, self.N, "U")[0] if U is not None else None
        fp = _dev_ptr(f, self.N, "f")[0] if f is not None else None
        fn = load().ert_vie_transport_noalloc if noalloc else load().ert_vie_transport
        _check(fn(self.handle, up, fp, dirs.ctypes.data_as(_dp), nd, pp),
               "ert_vie_transport_noalloc" if noalloc else "ert_vie_transport")
        return phi

    def net_apply(self, net, r, z):
        """z = M(r): the learned preconditioner `net` (on this grid or a coarsened one) as the
        solver applies it, on this plan's media (r, z: (N,) float64 CUDA tensors)."""
        rp, nr = _dev_ptr(r, self.N, "r")
        zp, nz = _dev_ptr(z, self.N, "z")
        if nr != 1 or nz != 1:
            raise ValueError("one column")
        _check(load().ert_vie_net_apply(self.handle, net.handle, rp, zp), "ert_vie_net_apply")
        return z

    def restrict(self, x, y, factor):
        """y = cell averages of x over factor^3 blocks (x: (nrhs, N) or (N,) float64 CUDA tensor
        on this grid, y: the same on the grid coarsened by factor)."""
        xp, nx = _dev_ptr(x, self.N, "x")
        nc = self.N // factor ** 3
        yp, ny = _dev_ptr(y, nc, "y")
        if nx != ny:
            raise ValueError("x and y differ in nrhs")
        _check(load().ert_vie_restrict(self.handle, int(factor), xp, yp, nx), "ert_vie_restrict")
        return y

    def diff_precond(self, r, z):
        """z = r + (two V-cycles for the diffusion approximation with source sigma_s r)."""
        rp, nr = _dev_ptr(r, self.N, "r")
        zp, nz = _dev_ptr(z, self.N, "z")
        if nr != nz:
            raise ValueError("r and z differ in nrhs")
        _check(load().ert_vie_diff_precond(self.handle, rp, zp, nr), "ert_vie_diff_precond")
        return z

    def fft_info(self):
        inf = FftInfo()
        _check(load().ert_vie_fft_info(self.handle, ctypes.byref(inf)), "ert_vie_fft_info")
        return {"m": list(inf.m), "sigma_t_mean": inf.sigma_t_mean, "sigma_s_mean": inf.sigma_s_mean,
                "self_cell": inf.self_cell, "symbol_min": inf.symbol_min, "symbol_max": inf.symbol_max,
                "bytes": inf.bytes}

    def solve(self, f, U, tol=1e-8, max_iter=500, restart=0, mixed=False, inner_tol=1e-5, rhs_is_phi=False,
              allow_noconv=False, block=False, precond=None, precond_steps=0, history=None, precond_fft=False,
              precond_diffusion=False):
        """Algorithm 1 steps S.1-S.2.  precond: a Net (learned right preconditioner);
        precond_fft / precond_diffusion: right-precondition by the FFT-based preconditioner of
        the mean medium, or by the diffusion preconditioner (with precond, the network acts on
        its output);
        history: float64 CUDA tensor (2k, N) receiving (U_k, r_k) of the plain solve's cycles."""
        fp, nf = _dev_ptr(f, self.N, "f")
        up, nu = _dev_ptr(U, self.N, "U")
        if nf != nu:
            raise ValueError("f and U differ in nrhs")
        so = SolveOpts()
        so.tol = float(tol)
        so.max_iter = int(max_iter)
        so.restart = int(restart)
        so.mixed = 1 if mixed else 0
        so.inner_tol = float(inner_tol)
        so.rhs_is_phi = 1 if rhs_is_phi else 0
        so.block = 1 if block else 0
        so.precond_steps = int(precond_steps)
        if precond_fft and precond_diffusion:
            raise ValueError("choose one fixed preconditioner")
        so.precond_kind = PRECOND_FFT if precond_fft else (PRECOND_DIFFUSION if precond_diffusion else PRECOND_NONE)
        if precond is not None:
            so.precond = precond.handle.value
        if history is not None:
            hp, hn = _dev_ptr(history, self.N, "history")
            if hn % 2:
                raise ValueError("history needs an even number of rows (iterate, residual)")
            so.history = hp
            so.history_max = hn // 2
        info = SolveInfo()
        st = load().ert_vie_solve(self.handle, fp, up, nf, ctypes.byref(so), ctypes.byref(info))
        out = {k: getattr(info, k) for k, _ in SolveInfo._fields_}
        out["status"] = st
        if not (st == OK or (allow_noconv and st == ENOCONV)):
            _check(st, "ert_vie_solve")
        return out

    def profile(self, enable):
        """Toggle per-stage event timing; returns {stage: (ms, launches)} recorded so far."""
        ms = (ctypes.c_double * NSTAGES)()
        ln = (ctypes.c_int * NSTAGES)()
        _check(load().ert_vie_profile(self.handle, int(bool(enable)), ms, ln), "ert_vie_profile")
        return {STAGES[i]: (ms[i], ln[i]) for i in range(NSTAGES)}

    def fmm_info(self, prec=None):
        p = self.opts.prec if prec is None else (_PREC[prec] if isinstance(prec, str) else prec)
        inf = FmmInfo()
        _check(load().ert_vie_fmm_info(self.handle, int(p), ctypes.byref(inf)), "ert_vie_fmm_info")
        L = inf.levels
        return {"levels": L, "leaf": inf.leaf, "cheb_n": inf.cheb_n, "nodes": inf.nodes,
                "nodes_padded": inf.nodes_padded, "rank": [inf.rank[l] for l in range(L + 1)],
                "far_pairs": [inf.far_pairs[l] for l in range(L + 1)], "near_pairs": inf.near_pairs,
                "form_near": inf.form_near, "form_far": [inf.form_far[l] for l in range(L + 1)],
                "near_table": inf.near_table, "far_rebuilt": [inf.far_rebuilt[l] for l in range(L + 1)],
                "cache_bytes": inf.cache_bytes}

    def diag(self):
        d = np.empty(self.N)
        _check(load().ert_vie_diag(self.handle, d.ctypes.data_as(_dp)), "ert_vie_diag")
        return d

    def size(self):
        return int(load().ert_vie_size(self.handle))

    def close(self):
        if self._h is not None and self._h.value:
            load().ert_vie_destroy(self._h)
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_from_case(case, method="direct", prec="fp64", cheb_n=0, leaf=0, nrhs_max=1, stream=None, svd_tol=0.0,
                   inner_cheb_n=0, inner_near16=False, scheme=0, form=None, far_cache_gb=0.0):
    return Plan(case["dim"], case["n"], case["h"], case["sigma_t"], case["sigma_s"], kernel=case["kernel"],
                method=method, prec=prec, cheb_n=cheb_n, leaf=leaf, nrhs_max=nrhs_max, stream=stream,
                svd_tol=svd_tol, inner_cheb_n=inner_cheb_n, inner_near16=inner_near16, scheme=scheme, form=form,
                far_cache_gb=far_cache_gb)


def _load_net():
    L = load()
    if getattr(L, "_net_ready", False):
        return L
    L.ert_net_param_count.restype = ctypes.c_long
    L.ert_net_param_count.argtypes = [ctypes.POINTER(NetOpts)]
    L.ert_net_create.restype = ctypes.c_int
    L.ert_net_create.argtypes = [ctypes.POINTER(NetOpts), _vp, ctypes.POINTER(_vp)]
    L.ert_net_size.restype = ctypes.c_long
    L.ert_net_size.argtypes = [_vp]
    L.ert_net_set_params.restype = ctypes.c_int
    L.ert_net_set_params.argtypes = [_vp, ctypes.POINTER(ctypes.c_float)]
    L.ert_net_get_params.restype = ctypes.c_int
    L.ert_net_get_params.argtypes = [_vp, ctypes.POINTER(ctypes.c_float)]
    L.ert_net_forward.restype = ctypes.c_int
    L.ert_net_forward.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int]
    L.ert_net_grad.restype = ctypes.c_int
    L.ert_net_grad.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, _dp, ctypes.POINTER(ctypes.c_float)]
    L.ert_net_train_step.restype = ctypes.c_int
    L.ert_net_train_step.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.POINTER(NetTrainOpts), _dp]
    L.ert_net_destroy.restype = None
    L.ert_net_destroy.argtypes = [_vp]
    L._net_ready = True
    return L


class Net:
    """The learned right preconditioner (ert_net_*): a 3D U-Net on an n0 x n1 x n2 grid.

    Vectors are float64 CUDA tensors (N,) or (batch, N); forward/grad/train take one
    medium per column (sigma_t, sigma_s of the same shape as r)."""

    def __init__(self, n, batch_max=1, widths=(16, 32, 64), stream=None):
        L = _load_net()
        o = NetOpts()
        o.dim = 3
        for a in range(3):
            o.n[a] = int(n[a])
            o.width[a] = int(widths[a])
        o.batch_max = int(batch_max)
        self.opts = o
        self.n = tuple(int(v) for v in n)
        self.N = int(np.prod(self.n))
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        sp = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        h = _vp()
        _check(L.ert_net_create(ctypes.byref(o), sp, ctypes.byref(h)), "ert_net_create")
        self._h = h
        self.size = int(L.ert_net_size(h))

    @staticmethod
    def param_count(widths=(16, 32, 64)):
        o = NetOpts()
        o.dim = 3
        for a in range(3):
            o.width[a] = int(widths[a])
        return int(_load_net().ert_net_param_count(ctypes.byref(o)))

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise RuntimeError("network is closed")
        return self._h

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32).reshape(-1)
        if p.size != self.size:
            raise ValueError("expected %d parameters, got %d" % (self.size, p.size))
        _check(_load_net().ert_net_set_params(self.handle, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "ert_net_set_params")

    def get_params(self):
        p = np.empty(self.size, dtype=np.float32)
        _check(_load_net().ert_net_get_params(self.handle, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "ert_net_get_params")
        return p

    def _vecs(self, **kw):
        ptrs, nb = [], None
        for name, t in kw.items():
            ptr, b = _dev_ptr(t, self.N, name)
            if nb is not None and b != nb:
                raise ValueError("batch sizes differ")
            nb = b
            ptrs.append(ptr)
        return ptrs, nb

    def forward(self, r, sigma_t, sigma_s, z):
        (rp, sp, ssp, zp), b = self._vecs(r=r, sigma_t=sigma_t, sigma_s=sigma_s, z=z)
        _check(_load_net().ert_net_forward(self.handle, rp, sp, ssp, zp, b), "ert_net_forward")
        return z

    def grad(self, r, e, sigma_t, sigma_s):
        (rp, ep, sp, ssp), b = self._vecs(r=r, e=e, sigma_t=sigma_t, sigma_s=sigma_s)
        loss = ctypes.c_double()
        g = np.empty(self.size, dtype=np.float32)
        _check(_load_net().ert_net_grad(self.handle, rp, ep, sp, ssp, b, ctypes.byref(loss),
                                        g.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), "ert_net_grad")
        return loss.value, g

    def train_step(self, r, e, sigma_t, sigma_s, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, want_loss=True):
        (rp, ep, sp, ssp), b = self._vecs(r=r, e=e, sigma_t=sigma_t, sigma_s=sigma_s)
        o = NetTrainOpts(float(lr), float(beta1), float(beta2), float(eps))
        loss = ctypes.c_double()
        _check(_load_net().ert_net_train_step(self.handle, rp, ep, sp, ssp, b, ctypes.byref(o),
                                              ctypes.byref(loss) if want_loss else None), "ert_net_train_step")
        return loss.value if want_loss else None

    def close(self):
        if self._h is not None and self._h.value:
            _load_net().ert_net_destroy(self._h)
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
