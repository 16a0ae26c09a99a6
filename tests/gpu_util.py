"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI on
torch-allocated device memory and compare with the oracle."""
import numpy as np


def torch_dev():
    import torch
    return torch


def to_dev(a):
    """Host (N,) or (N, nrhs) float64 -> contiguous CUDA tensor (N,) or (nrhs, N)."""
    torch = torch_dev()
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 2:
        a = np.ascontiguousarray(a.T)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_host(t):
    torch = torch_dev()
    torch.cuda.synchronize()
    a = t.detach().cpu().numpy()
    if a.ndim == 2:
        a = np.asfortranarray(a.T)
    return a


def gpu_apply(plan, x, op, method=None, prec=None):
    torch = torch_dev()
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    plan.apply(xd, yd, op=op, method=method, prec=prec)
    return to_host(yd)


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_problem(O, case, sigma_s=None):
    return O.Problem(case["dim"], case["n"], case["h"], case["kernel"], case["sigma_t"],
                     case["sigma_s"] if sigma_s is None else sigma_s)


def log(*msg):
    print(*msg, flush=True)
