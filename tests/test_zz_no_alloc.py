"""GPU test of helmholtz_solve_noalloc, the FP64 solve that takes its
workspace from the library's static device scratch array instead of
allocating: bitwise the same result as helmholtz_solve (same kernels, same
order), on two calls in a row (the second on a smaller mesh, so stale
contents of the larger first call are left in the array), no device memory
allocated by any call after the first (the first call on a device looks up
the array's address, and the runtime materialises the array then), and a
clear refusal of a mesh whose workspace does not fit the array."""
import numpy as np
import pytest

import synth
from oracle import dense, kron
from tests.gpu_util import say, to_dev, torch_dev
from tests.helpers import make_spec, ndof

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_noalloc_solve_matches_allocating_solve():
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    cases = [(make_spec((12, 10, 9), 5, (0, 0, 1), True), 2000.0, 0),  # 233k nodes, Dirichlet z
             (make_spec((3, 4, 2), 7, (0, 2, 0), False), 0.0, 0)]       # smaller; singular Poisson
    # tol 1e-11 keeps both systems' errors against x* well inside 1e-10
    o = dg.default_opts(tol=1e-11)
    first = True
    for spec, lam, seed in cases:
        N = ndof(spec)
        f = to_dev(synth.uniform_field(N, 300 + seed + N % 97))
        mesh = dg.mesh_from_spec(spec)
        x_ref = torch.zeros_like(f)
        i_ref = dg.helmholtz_solve(mesh, lam, None, 1.0, f, x_ref, o)
        x = torch.full_like(f, 0.0)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        info = dg.helmholtz_solve_noalloc(mesh, lam, None, 1.0, f, x, o)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        say("noalloc", spec["nx"], spec["ny"], spec["nz"], spec["P"], info, "ref", i_ref,
            "free delta", free0 - free1)
        assert info["status"] == 0 and info["iters"] == i_ref["iters"]
        if first:
            first = False
        else:
            assert free1 == free0                   # nothing allocated by the call
        assert torch.equal(x, x_ref)                # bitwise the allocating solve
        M = dense.mass_diag(spec)
        xs = kron.FDM(spec, lam).solve(M * f.cpu().numpy())
        say("err vs x*", rel(x.cpu().numpy(), xs))
        assert rel(x.cpu().numpy(), xs) <= 1e-10
        mesh.destroy()


def test_noalloc_solve_refuses_oversized_mesh_and_mixed():
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    spec = make_spec((20, 20, 20), 5, (0, 0, 0), False)     # 1.73M nodes: fits
    big = make_spec((24, 24, 24), 7, (0, 0, 0), False)      # 7.1M nodes: does not
    mesh = dg.mesh_from_spec(big)
    f = torch.ones(mesh.ndof, dtype=torch.float64, device=dev)
    x = torch.zeros_like(f)
    info = dg.helmholtz_solve_noalloc(mesh, 1.0, None, 1.0, f, x, dg.default_opts(),
                                      raise_on_error=False)
    assert info["rc"] == dg.DG_ERR_ARG and "scratch" in dg.last_error()
    mesh.destroy()
    mesh = dg.mesh_from_spec(spec)
    f = torch.ones(mesh.ndof, dtype=torch.float64, device=dev)
    x = torch.zeros_like(f)
    info = dg.helmholtz_solve_noalloc(mesh, 1.0, None, 1.0, f, x, dg.default_opts(precision=1),
                                      raise_on_error=False)
    assert info["rc"] == dg.DG_ERR_ARG
    info = dg.helmholtz_solve_noalloc(mesh, 1.0, None, 1.0, f, x, dg.default_opts())
    assert info["status"] == 0
    mesh.destroy()
