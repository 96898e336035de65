"""The divergence and gradient kernels' phases (the projection's P / P-1 pair
and the equal-order pair of the viscous terms) run on the CPU, for every
thread index of a work-group in turn (tests/host_phases), built with an
address sanitizer on the host side: their LDS and global indexing stays in
bounds, and their results equal the oracle's definitions (<= 1e-12 relative,
the same exactly integrated sums in FP64) on every degree the kernels take,
periodic, Dirichlet and Neumann axes, single-element periodic axes, a graded
axis, with and without wall data."""
import os
import subprocess

import numpy as np
import pytest

from oracle import gll, projection
from tests.helpers import make_spec, ndof

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CASES = [((2, 2, 2), 4, (0, 0, 0), False),
         ((3, 2, 2), 5, (0, 0, 1), True),
         ((1, 3, 2), 6, (0, 1, 2), False),
         ((2, 1, 3), 7, (2, 0, 1), True),
         ((2, 2, 1), 8, (1, 2, 0), False),
         ((1, 1, 1), 7, (0, 0, 0), False),
         ((3, 2, 2), 7, (1, 1, 1), True)]
IDS = ["P4_periodic", "P5_channel", "P6_n1x", "P7_mixed", "P8_n1z", "P7_one_element", "P7_walls"]


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("phases") / "projection_phases")
    cmd = [HIPCC, "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
           "-Xarch_host", "-fsanitize=address",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2112_04167_amd", "csrc"),
           os.path.join(HERE, "host_phases", "projection_phases.hip"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def gll_mass(spec):
    """Diagonal of the GLL mass in the ABI layout: J w_a w_b w_c."""
    P = spec["P"]
    w = gll.weights(P)
    hx, hy, hz = (np.diff(np.asarray(spec[k], dtype=np.float64)) for k in ("xv", "yv", "zv"))
    J = (hz[:, None, None] * hy[None, :, None] * hx[None, None, :]) / 8.0
    wn = w[:, None, None] * w[None, :, None] * w[None, None, :]  # [c][b][a]
    return (J[:, :, :, None, None, None] * wn[None, None, None]).ravel()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def run_case(harness, tmp_path, case, with_vb, equal):
    n, P, bc, st = case
    spec = make_spec(n, P, bc, st)
    N = ndof(spec)
    Nq = N if equal else n[0] * n[1] * n[2] * P ** 3
    rng = np.random.default_rng(11 + P)
    v = [rng.uniform(-1, 1, N) for _ in range(3)]
    vb = [rng.uniform(-1, 1, N) for _ in range(3)] if with_vb else []
    psi = np.random.default_rng(23 + P).uniform(-1, 1, Nq)
    fac = [np.random.default_rng(31 + P).uniform(0.5, 2.0, N)] if equal else []
    h = [np.diff(np.asarray(spec[k], dtype=np.float64)) for k in ("xv", "yv", "zv")]
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    np.concatenate(h + v + vb + [psi] + fac).astype(np.float64).tofile(fin)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([harness, str(P), *map(str, n), *map(str, bc), str(int(with_vb)), str(int(equal)),
                        str(fin), str(fout)], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    out = np.fromfile(fout)
    extra = N if equal else 0
    assert out.size == Nq + extra + 3 * N
    q_degree = P if equal else None
    div = out[:Nq]
    want_div = projection.divergence(spec, v, vb or None, q_degree=q_degree)
    assert rel(div, want_div) <= 1e-12
    if equal:
        # the nodal form: the weak vector over the diagonal GLL mass
        # J w_a w_b w_c, times the nodal factor
        assert rel(out[Nq:Nq + N], want_div / gll_mass(spec) * fac[0]) <= 1e-12
    want = projection.gradient(spec, psi, q_degree=q_degree)
    for d in range(3):
        g = out[Nq + extra + d * N:Nq + extra + (d + 1) * N]
        assert rel(g, want[d] * fac[0] if equal else want[d]) <= 1e-12


@pytest.mark.parametrize("case", CASES, ids=IDS)
@pytest.mark.parametrize("with_vb", [False, True])
def test_projection_phases_match_oracle(harness, tmp_path, case, with_vb):
    run_case(harness, tmp_path, case, with_vb, False)


EQ_CASES = [((2, 2, 2), 3, (0, 0, 0), False)] + CASES
EQ_IDS = ["P3_periodic"] + IDS


@pytest.mark.parametrize("case", EQ_CASES, ids=EQ_IDS)
@pytest.mark.parametrize("with_vb", [False, True])
def test_equal_order_phases_match_oracle(harness, tmp_path, case, with_vb):
    """The equal-order pair (F_d2, F_d3): scalar degree P, the gradient with a
    nodal factor."""
    run_case(harness, tmp_path, case, with_vb, True)
