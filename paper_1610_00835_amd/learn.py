"""Training of the learned right preconditioner (ert_net_* in include/ertvie.h).

Training pairs come from the method's own solves: a plain restarted GMRES solve
of (I - K) U = phi records, at the start of every cycle k, the iterate U_k and
its residual r_k = phi - (I - K) U_k; once converged, the correction of U_k is
e_k = U - U_k, and (I - K) e_k = r_k up to the solve tolerance.  The network
learns r -> e on those pairs (with the medium as extra input channels); a network on
a coarser grid learns the cell averages of the pairs (restrict_pairs).

All arithmetic of the solve and of training runs in libertvie.so; this module
draws the seeded initial parameters and batches, and copies vectors between
torch tensors (device memory plumbing).
"""
import numpy as np

from . import ertvie


def init_params(widths=(16, 32, 64), seed=0):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, FP32, canonical layout."""
    w1, w2, w3 = widths
    shapes = [(w1, 3, 3), (w1, w1, 3), (w2, w1, 3), (w2, w2, 3), (w3, w2, 3), (w3, w3, 3),
              (w2, w3 + w2, 3), (w2, w2, 3), (w1, w2 + w1, 3), (w1, w1, 3), (1, w1, 1)]
    rng = np.random.default_rng(seed)
    out = []
    for co, ci, k in shapes:
        fan_in = ci * k ** 3
        out.append(rng.standard_normal(co * ci * k ** 3) * np.sqrt(2.0 / fan_in))
        out.append(np.zeros(co))
    return np.concatenate(out).astype(np.float32)


def collect_pairs(plan, f, restart=5, tol=1e-10, max_pairs=64, max_iter=3000, fft=False):
    """Solve (I - K) U = A f with plain restarted GMRES and return (R, E, info): residuals
    r_k and corrections e_k = U - U_k of the cycles, as (k, N) float64 CUDA tensors.
    With fft, R holds M r_k instead (M the FFT-based preconditioner of the mean medium):
    the input a network sees when it acts on that preconditioner's output."""
    import torch
    N = plan.N
    fd = torch.as_tensor(np.ascontiguousarray(f, dtype=np.float64)).cuda()
    U = torch.empty_like(fd)
    hist = torch.empty((2 * max_pairs, N), dtype=torch.float64, device="cuda")
    info = plan.solve(fd, U, tol=tol, max_iter=max_iter, restart=restart, history=hist, allow_noconv=True)
    k = info["history_count"]
    Uk = hist[0:2 * k:2]
    R = hist[1:2 * k:2].clone()
    E = (U.unsqueeze(0) - Uk).contiguous()
    if fft:
        for i in range(k):
            plan.fft_precond(R[i], R[i])
    return R, E, info


def restrict_pairs(plan, R, E, sigma_t, sigma_s, f):
    """The pairs (R, E) and the medium of `plan` averaged over f^3 blocks (ert_vie_restrict):
    the training data of a network on the plan's grid coarsened by f.  Returns (Rc, Ec,
    sigma_t_c, sigma_s_c), the media as host arrays."""
    import torch
    nc = plan.N // f ** 3
    Rc = torch.empty((R.shape[0], nc), dtype=torch.float64, device="cuda")
    Ec = torch.empty_like(Rc)
    plan.restrict(R.contiguous(), Rc, f)
    plan.restrict(E.contiguous(), Ec, f)
    med = torch.as_tensor(np.stack([np.asarray(sigma_t, dtype=np.float64), np.asarray(sigma_s, dtype=np.float64)])).cuda()
    medc = torch.empty((2, nc), dtype=torch.float64, device="cuda")
    plan.restrict(med, medc, f)
    torch.cuda.synchronize()
    mc = medc.cpu().numpy()
    return Rc, Ec, mc[0], mc[1]


class PairSet:
    """Pairs (r, e) with the medium of each pair, resident on the GPU."""

    def __init__(self):
        self.R, self.E, self.ST, self.SS = [], [], [], []

    def add(self, R, E, sigma_t, sigma_s):
        import torch
        k = R.shape[0]
        st = torch.as_tensor(np.ascontiguousarray(sigma_t, dtype=np.float64)).cuda()
        ss = torch.as_tensor(np.ascontiguousarray(sigma_s, dtype=np.float64)).cuda()
        self.R.append(R)
        self.E.append(E)
        self.ST.append(st.unsqueeze(0).expand(k, -1))
        self.SS.append(ss.unsqueeze(0).expand(k, -1))

    def finalize(self):
        import torch
        self.R = torch.cat(self.R).contiguous()
        self.E = torch.cat(self.E).contiguous()
        self.ST = torch.cat(self.ST).contiguous()
        self.SS = torch.cat(self.SS).contiguous()
        return self

    def __len__(self):
        return int(self.R.shape[0])


def train(net, pairs, steps, batch=4, lr=1e-3, seed=0, lr_final=None, log_every=0, log=None):
    """Adam on random minibatches of `pairs`; the step size decays linearly to lr_final
    (default lr / 10).  Returns the list of minibatch losses."""
    import torch
    rng = np.random.default_rng(seed)
    n = len(pairs)
    lr_final = lr / 10 if lr_final is None else lr_final
    losses = []
    for s in range(steps):
        idx = torch.as_tensor(rng.choice(n, size=batch, replace=n < batch), device="cuda")
        a = lr + (lr_final - lr) * s / max(1, steps - 1)
        want = log_every > 0 and (s % log_every == 0 or s == steps - 1)
        L = net.train_step(pairs.R[idx].contiguous(), pairs.E[idx].contiguous(), pairs.ST[idx].contiguous(),
                           pairs.SS[idx].contiguous(), lr=a, want_loss=want)
        if want:
            losses.append((s, L))
            if log:
                log("step %d lr %.2e loss %.4f" % (s, a, L))
    return losses
