"""Shared helpers of the GPU parity tests."""
import sys

import numpy as np


def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch, torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    torch, dev = torch_dev()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)


def gpu_apply(spec, lam, nu, x, precision=0):
    """y = A x on the GPU through the C-ABI; nu scalar or nodal array."""
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    dt = torch.float64 if precision == dg.DG_FP64 else torch.float32
    mesh = dg.mesh_from_spec(spec)
    xd = to_dev(x, dt)
    yd = torch.empty_like(xd)
    nud = None if np.isscalar(nu) else to_dev(nu, dt)
    dg.helmholtz_apply(mesh, lam, nud, nu if np.isscalar(nu) else 0.0, xd, yd, precision)
    torch.cuda.synchronize()
    y = yd.double().cpu().numpy()
    mesh.destroy()
    return y
