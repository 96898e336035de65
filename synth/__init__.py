"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the method: only vertex arrays of the
Cartesian meshes, seeded random numbers, and the workload descriptions.  Both
the oracle side and the GPU side receive the very same arrays from here.

Workloads (the implicit-stage problems of arXiv 2112.04167, Alg. 3: a
Helmholtz problem lambda*u - div(nu grad u) = f per velocity component and a
pressure Poisson problem, on hexahedral GLL meshes, Sec. 3.3):

  small_periodic   4^3 elements, P=4, periodic, lambda=nu=1, manufactured RHS
  stretched_large  32^3 elements, P=7, tanh-stretched in z (factor 1.5),
                   Dirichlet z, periodic x,y; lambda=1/(0.4358665*dt*nu) with
                   dt=nu=1e-3 and unit nu in the operator; uniform random RHS
                   (plus the pressure Poisson problem: lambda=0, mean-zero RHS)
  mixed_small      the small_periodic mesh at P=7, lambda in {1e2,1e4,1e6}
  batched_channel  24^3, P=5, periodic x,y, Dirichlet z (velocity), Neumann z
                   (pressure); nu(x)=1e-3(1+0.5 sin(2 pi x) cos(2 pi y))
  vvp_large        16^3 elements, P=7, periodic on [-1/2,1/2]^3: the VVP
                   vortex array with nu(v) = 0.01 + 0.01 (|v|/2)^2 (one full
                   IMEX-RK step, Alg. 3)
  serving_stream   2000 requests, Poisson arrivals at 200/s, n^3 cubes,
                   n~U{6..40}, P~U{3..8}, lambda log-uniform in [1,1e6],
                   20% Poisson (lambda=0)
"""
import math

import numpy as np

BC_PERIODIC, BC_DIRICHLET, BC_NEUMANN = 0, 1, 2

# the SDIRK diagonal coefficient and step used for the large Helmholtz case
SDIRK_GAMMA = 0.4358665
DT_LARGE = 1e-3
NU_PHYS_LARGE = 1e-3


def vertices_uniform(n, lo=0.0, hi=1.0):
    """n+1 equispaced vertices on [lo, hi]."""
    v = lo + (hi - lo) * np.arange(n + 1, dtype=np.float64) / n
    v[-1] = hi
    return v


def vertices_tanh(n, beta=1.5):
    """n+1 vertices on [0,1] clustered toward both ends:
    z_k = (1 + tanh(beta (2k/n - 1)) / tanh(beta)) / 2."""
    k = np.arange(n + 1, dtype=np.float64)
    v = 0.5 * (1.0 + np.tanh(beta * (2.0 * k / n - 1.0)) / np.tanh(beta))
    v[0], v[-1] = 0.0, 1.0
    return v


def uniform_field(ndof, seed, lo=-1.0, hi=1.0, dtype=np.float64):
    """f ~ U[lo, hi] from NumPy's PCG64 with a fixed seed, in ABI layout."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=ndof).astype(dtype)


def splitmix64_uniform(n, seed):
    """f_i = 2 (z_i >> 11) / 2^53 - 1 with z_i the (i+1)-th output of
    SplitMix64 (Steele, Lea & Flood 2014) started from `seed` -- the
    counter-based generator the request server uses on the device."""
    gamma = np.uint64(0x9E3779B97F4A7C15)
    i = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + i * gamma
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return 2.0 * ((z >> np.uint64(11)).astype(np.float64) / 9007199254740992.0) - 1.0


def ndof(n, P):
    return n[0] * n[1] * n[2] * (P + 1) ** 3


def mesh_spec(name):
    """Mesh description: dict(nx, ny, nz, P, xv, yv, zv, bc)."""
    if name == "small_periodic":
        n, P = 4, 4
        return dict(nx=n, ny=n, nz=n, P=P, xv=vertices_uniform(n), yv=vertices_uniform(n),
                    zv=vertices_uniform(n), bc=(BC_PERIODIC,) * 3)
    if name == "mixed_small":
        n, P = 4, 7
        return dict(nx=n, ny=n, nz=n, P=P, xv=vertices_uniform(n), yv=vertices_uniform(n),
                    zv=vertices_uniform(n), bc=(BC_PERIODIC,) * 3)
    if name == "stretched_large":
        n, P = 32, 7
        return dict(nx=n, ny=n, nz=n, P=P, xv=vertices_uniform(n), yv=vertices_uniform(n),
                    zv=vertices_tanh(n, 1.5), bc=(BC_PERIODIC, BC_PERIODIC, BC_DIRICHLET))
    if name == "vvp_large":
        # the VVP vortex array at scale: [-1/2, 1/2]^3, periodic, 16^3 elements
        # of degree 7 (2.1M nodes per velocity component, pressure degree 6)
        n, P = 16, 7
        v = vertices_uniform(n, -0.5, 0.5)
        return dict(nx=n, ny=n, nz=n, P=P, xv=v, yv=v.copy(), zv=v.copy(), bc=(BC_PERIODIC,) * 3)
    if name == "batched_channel":
        n, P = 24, 5
        return dict(nx=n, ny=n, nz=n, P=P, xv=vertices_uniform(n), yv=vertices_uniform(n),
                    zv=vertices_uniform(n), bc=(BC_PERIODIC, BC_PERIODIC, BC_DIRICHLET))
    raise KeyError(name)


def scaled_mesh_spec(name, n, P=None, zstretch=None):
    """A smaller copy of a named mesh (same BCs / grading), n elements per axis."""
    s = mesh_spec(name)
    P = s["P"] if P is None else P
    zv = vertices_tanh(n, 1.5) if (zstretch if zstretch is not None else name == "stretched_large") \
        else vertices_uniform(n)
    return dict(nx=n, ny=n, nz=n, P=P, xv=vertices_uniform(n), yv=vertices_uniform(n), zv=zv,
                bc=s["bc"])


def large_helmholtz_lambda():
    """lambda = 1/(gamma dt nu) for the large stretched Helmholtz case."""
    return 1.0 / (SDIRK_GAMMA * DT_LARGE * NU_PHYS_LARGE)


def batched_lambda():
    """lambda = 1/(gamma dt) for the batched velocity systems (physical nu in the operator)."""
    return 1.0 / (SDIRK_GAMMA * DT_LARGE)


SEEDS = dict(large_helmholtz=21120, large_poisson=41670, mixed=3,
             batched_velocity=(41, 42, 43), batched_pressure=44, serving_master=5,
             serving_base=5000)


def serving_stream(nreq=2000, rate=200.0, seed=SEEDS["serving_master"], nmin=6, nmax=40,
                   Pmin=3, Pmax=8, p_poisson=0.2, lam_lo=1.0, lam_hi=1e6):
    """Request list for the serving workload.

    Each request: dict(id, t_arrival [s], n, P, poisson, lam, rhs_seed).
    Arrivals are a Poisson process (exponential gaps with mean 1/rate)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=nreq)
    t = np.cumsum(gaps) - gaps[0]
    ns = rng.integers(nmin, nmax + 1, size=nreq)
    Ps = rng.integers(Pmin, Pmax + 1, size=nreq)
    pois = rng.uniform(size=nreq) < p_poisson
    loglam = rng.uniform(math.log10(lam_lo), math.log10(lam_hi), size=nreq)
    out = []
    for i in range(nreq):
        out.append(dict(id=i, t_arrival=float(t[i]), n=int(ns[i]), P=int(Ps[i]),
                        poisson=bool(pois[i]), lam=0.0 if pois[i] else float(10.0 ** loglam[i]),
                        rhs_seed=SEEDS["serving_base"] + i))
    return out


# ----------------------------------------------------------------------------
# The 3D vortex array with velocity-dependent viscosity (test case VVP of
# arXiv 2112.04167, Sec. 4.2): exact velocity and pressure on
# [-1/2, 1/2]^3, periodic, and the forcing that makes them a solution of the
# momentum equation with nu(v) = nu0 + nu1 (|v| / v_max)^2, v_max = 2.  The
# forcing is problem data: written from the closed-form derivatives of the
# exact solution (each velocity term is a product of two sines/cosines of
# 2 pi (x_k + t), so its Laplacian is -8 pi^2 times itself and d/dt is the
# sum of the three space derivatives).

VVP_VMAX = 2.0


def _vvp_parts(X, Y, Z, t, xp=np):
    k = 2.0 * np.pi
    sx, cx = xp.sin(k * (X + t)), xp.cos(k * (X + t))
    sy, cy = xp.sin(k * (Y + t)), xp.cos(k * (Y + t))
    sz, cz = xp.sin(k * (Z + t)), xp.cos(k * (Z + t))
    v = [(sx + cy) * sz, (cx + sy) * sz, (cx + cy) * cz]
    # J[i][m] = d v_i / d x_m
    J = [[k * cx * sz, -k * sy * sz, k * (sx + cy) * cz],
         [-k * sx * sz, k * cy * sz, k * (cx + sy) * cz],
         [-k * sx * cz, -k * sy * cz, -k * (cx + cy) * sz]]
    gp = [k * cx * sy * sz, k * sx * cy * sz, k * sx * sy * cz]
    return v, J, gp


def vvp_velocity(X, Y, Z, t, xp=np):
    """Exact VVP velocity (three arrays) at time t (xp: numpy or torch)."""
    return _vvp_parts(X, Y, Z, t, xp)[0]


def vvp_pressure(X, Y, Z, t):
    k = 2.0 * np.pi
    return np.sin(k * (X + t)) * np.sin(k * (Y + t)) * np.sin(k * (Z + t))


def vvp_forcing(X, Y, Z, t, nu0, nu1, vmax=VVP_VMAX, xp=np):
    """f = d_t v + div(v v) - div(nu(v) (grad v + grad v^T)) + grad p for the
    exact VVP fields (div v = 0); xp: numpy or torch."""
    v, J, gp = _vvp_parts(X, Y, Z, t, xp)
    nu = nu0 + nu1 * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2) / (vmax * vmax)
    dnu = [2.0 * nu1 / (vmax * vmax) * sum(v[m] * J[m][k] for m in range(3)) for k in range(3)]
    lap = -8.0 * np.pi ** 2
    f = []
    for i in range(3):
        dt_v = J[i][0] + J[i][1] + J[i][2]
        conv = sum(v[k] * J[i][k] for k in range(3))
        visc = sum(dnu[k] * (J[i][k] + J[k][i]) for k in range(3)) + nu * lap * v[i]
        f.append(dt_v + conv - visc + gp[i])
    return f


# A shear flow v = (u(y, t), 0, 0), u = sin(2 pi (y + t)), with the same
# viscosity law: divergence-free with no convective tendency (v.grad v = 0),
# so the momentum equation reduces to d_t u = d_y(nu(u) d_y u) + f_x.  The
# forcing below makes u the exact solution (problem data for the temporal
# order of the IMEX-RK step with an exact projection).

def shear_velocity(X, Y, Z, t, xp=np):
    u = xp.sin(2.0 * np.pi * (Y + t))
    return [u, 0.0 * u, 0.0 * u]


def shear_forcing(X, Y, Z, t, nu0, nu1, vmax=VVP_VMAX, xp=np):
    k = 2.0 * np.pi
    u = xp.sin(k * (Y + t))
    uy = k * xp.cos(k * (Y + t))
    nu = nu0 + nu1 * u * u / (vmax * vmax)
    nuy = 2.0 * nu1 * u * uy / (vmax * vmax)
    fx = uy - (nuy * uy - nu * k * k * u)     # d_t u = d_y u here
    return [fx, 0.0 * u, 0.0 * u]
