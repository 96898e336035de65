"""GPU parity of the sum-factorised SIP-DG apply and its Jacobi diagonal
against the oracle (naive matrix-free loop in FP64).

Tolerances: FP64, ||y_gpu - y_ref||_inf <= 1e-12 ||y_ref||_inf -- each output
is a sum of O(10 (P+1)) products of O(1) relative magnitude, so rounding
differences between the two summation orders stay within ~100 eps of the
row scale.  FP32: the reference is the FP64 oracle applied to the FP32-rounded
input, nu and geometry identical; the bound 2e-5 ||y||_inf is ~300 FP32 eps.
"""
import numpy as np
import pytest

import synth
from oracle import naive
from tests.gpu_util import gpu_apply, say, to_dev, torch_dev
from tests.helpers import make_spec, ndof, channel_nu

pytestmark = pytest.mark.gpu

# (elements, P, bc, z-stretch): ragged element counts for every work-group
# size, single-element periodic axes, all BC kinds
SHAPES = [
    ((3, 2, 3), 3, (0, 0, 0), False),
    ((3, 2, 3), 4, (0, 1, 2), True),
    ((2, 3, 2), 5, (1, 0, 1), True),
    ((3, 3, 1), 6, (2, 2, 0), False),
    ((3, 2, 3), 7, (0, 0, 1), True),
    ((2, 2, 2), 8, (1, 2, 0), True),
    ((1, 1, 1), 7, (0, 0, 0), False),
    ((1, 2, 1), 5, (0, 0, 1), False),
    ((5, 1, 2), 3, (1, 0, 2), True),
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "n%s_P%d_bc%s" % (s[0], s[1], s[2]))
@pytest.mark.parametrize("nodal", [False, True])
def test_apply_fp64_parity(shape, nodal):
    n, P, bc, st = shape
    spec = make_spec(n, P, bc, st)
    N = ndof(spec)
    rng = np.random.default_rng(11)
    x = rng.uniform(-1, 1, N)
    nu = rng.uniform(0.5, 2.0, N) if nodal else 1.7
    lam = 3.3
    say("apply fp64", shape, "nodal" if nodal else "const")
    y = gpu_apply(spec, lam, nu, x)
    yr = naive.Operator(spec, lam, nu).apply(x)
    assert np.abs(y - yr).max() <= 1e-12 * np.abs(yr).max()


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "n%s_P%d_bc%s" % (s[0], s[1], s[2]))
@pytest.mark.parametrize("nodal", [False, True])
def test_apply_fp32_parity(shape, nodal):
    n, P, bc, st = shape
    spec = make_spec(n, P, bc, st)
    # the FP32 path uses float element extents: give the oracle the same ones
    spec32 = dict(spec)
    for k in ("xv", "yv", "zv"):
        h = np.diff(spec[k]).astype(np.float32).astype(np.float64)
        spec32[k] = np.concatenate([[0.0], np.cumsum(h)])
    N = ndof(spec)
    rng = np.random.default_rng(12)
    x = rng.uniform(-1, 1, N).astype(np.float32)
    nu = rng.uniform(0.5, 2.0, N).astype(np.float32) if nodal else 1.25
    lam = 2.0
    say("apply fp32", shape, "nodal" if nodal else "const")
    y = gpu_apply(spec, lam, nu, x, precision=1)
    yr = naive.Operator(spec32, lam, nu if np.isscalar(nu) else nu.astype(np.float64)).apply(
        x.astype(np.float64))
    assert np.abs(y - yr).max() <= 2e-5 * np.abs(yr).max()


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "n%s_P%d_bc%s" % (s[0], s[1], s[2]))
def test_diag_parity(shape):
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    n, P, bc, st = shape
    spec = make_spec(n, P, bc, st)
    N = ndof(spec)
    rng = np.random.default_rng(13)
    nu = rng.uniform(0.5, 2.0, N)
    mesh = dg.mesh_from_spec(spec)
    for nuv in (1.3, nu):
        d = torch.empty(N, dtype=torch.float64, device=dev)
        dg.helmholtz_diag(mesh, 0.7, None if np.isscalar(nuv) else to_dev(nuv),
                          nuv if np.isscalar(nuv) else 0.0, d)
        torch.cuda.synchronize()
        dr = naive.Operator(spec, 0.7, nuv).diag()
        assert np.abs(d.cpu().numpy() - dr).max() <= 1e-13 * np.abs(dr).max()
    mesh.destroy()


def test_apply_bitwise_deterministic():
    spec = make_spec((3, 3, 3), 7, (0, 0, 1), True)
    x = synth.uniform_field(ndof(spec), 5)
    y1 = gpu_apply(spec, 2.0, 1.0, x)
    y2 = gpu_apply(spec, 2.0, 1.0, x)
    assert np.array_equal(y1, y2)


def test_apply_small_periodic_config():
    spec = synth.mesh_spec("small_periodic")
    x = synth.uniform_field(ndof(spec), 0)
    y = gpu_apply(spec, 1.0, 1.0, x)
    yr = naive.Operator(spec, 1.0, 1.0).apply(x)
    assert np.abs(y - yr).max() <= 1e-12 * np.abs(yr).max()


def test_apply_stretched_large_full_size():
    # the 32^3, P=7 tanh-stretched mesh (16.8M nodes) in the bench launch
    # configuration, compared over every node with the oracle
    spec = synth.mesh_spec("stretched_large")
    lam = synth.large_helmholtz_lambda()
    x = synth.uniform_field(ndof(spec), synth.SEEDS["large_helmholtz"])
    say("apply full size", ndof(spec))
    y = gpu_apply(spec, lam, 1.0, x)
    yr = naive.Operator(spec, lam, 1.0).apply(x)
    assert np.abs(y - yr).max() <= 1e-12 * np.abs(yr).max()
    # and with lambda = 0 (the Poisson operator of the same mesh)
    y0 = gpu_apply(spec, 0.0, 1.0, x)
    y0r = naive.Operator(spec, 0.0, 1.0).apply(x)
    assert np.abs(y0 - y0r).max() <= 1e-12 * np.abs(y0r).max()


def test_apply_batched_channel_nodal_nu_full_size():
    spec = synth.mesh_spec("batched_channel")
    nu = channel_nu(spec)
    lam = synth.batched_lambda()
    x = synth.uniform_field(ndof(spec), 41)
    y = gpu_apply(spec, lam, nu, x)
    yr = naive.Operator(spec, lam, nu).apply(x)
    assert np.abs(y - yr).max() <= 1e-12 * np.abs(yr).max()


def test_mesh_coordinates():
    import paper_2112_04167_amd as dg
    from tests.helpers import node_coords
    torch, dev = torch_dev()
    spec = make_spec((3, 2, 4), 5, (0, 1, 2), True)
    mesh = dg.mesh_from_spec(spec)
    X, Y, Z = [t.cpu().numpy() for t in dg.mesh_coordinates(mesh)]
    Xr, Yr, Zr = node_coords(spec)
    for a, b in ((X, Xr), (Y, Yr), (Z, Zr)):
        assert np.abs(a - b).max() <= 1e-15
    mesh.destroy()


@pytest.mark.parametrize("P", [3, 7])
@pytest.mark.parametrize("prec", [0, 1])
def test_apply_unaligned_vectors(P, prec):
    # at P = 3 and 7 aligned FP64 vectors take the 16-byte chunk path for the
    # own element and y; vectors offset by one value (not 16-byte aligned)
    # take the per-line path (as FP32 always does).  Both must agree with
    # each other bitwise (the same arithmetic per node) and with the oracle.
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    spec = make_spec((3, 2, 3), P, (0, 0, 1), True)
    N = ndof(spec)
    dt = torch.float64 if prec == 0 else torch.float32
    x = synth.uniform_field(N, 23)
    nuv = np.random.default_rng(3).uniform(0.5, 2.0, N)
    mesh = dg.mesh_from_spec(spec)
    for nu in (None, nuv):
        xa = torch.from_numpy(x).to(dev, dt)
        nua = None if nu is None else torch.from_numpy(nu).to(dev, dt)
        ya = torch.zeros(N, dtype=dt, device=dev)
        dg.helmholtz_apply(mesh, 2.5, nua, 1.3, xa, ya, precision=prec)
        big_x = torch.zeros(N + 1, dtype=dt, device=dev)
        big_y = torch.zeros(N + 1, dtype=dt, device=dev)
        big_x[1:] = xa
        nub = None
        if nua is not None:
            nub = torch.zeros(N + 1, dtype=dt, device=dev)
            nub[1:] = nua
        assert big_x[1:].data_ptr() % 16 != 0
        dg.helmholtz_apply(mesh, 2.5, None if nub is None else nub[1:], 1.3, big_x[1:], big_y[1:],
                           precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(ya, big_y[1:]), "chunked and per-line paths differ"
        if prec == 0:
            yr = naive.Operator(spec, 2.5, 1.3 if nu is None else nu).apply(x)
            assert np.abs(ya.cpu().numpy() - yr).max() <= 1e-12 * np.abs(yr).max()
    mesh.destroy()
