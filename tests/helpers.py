"""Test helpers: small meshes, node coordinates (from the oracle's GLL
nodes) and manufactured fields.  Used by the CPU pins and the GPU parity
tests alike; nothing here comes from the HIP path."""
import numpy as np

import synth
from oracle import gll


def make_spec(n, P, bc, zstretch=False, lo=0.0, hi=1.0):
    if np.isscalar(n):
        n = (n, n, n)
    return dict(nx=n[0], ny=n[1], nz=n[2], P=P,
                xv=synth.vertices_uniform(n[0], lo, hi), yv=synth.vertices_uniform(n[1], lo, hi),
                zv=synth.vertices_tanh(n[2], 1.5) if zstretch else synth.vertices_uniform(n[2], lo, hi),
                bc=tuple(bc))


def ndof(spec):
    return spec["nx"] * spec["ny"] * spec["nz"] * (spec["P"] + 1) ** 3


def node_coords(spec):
    """(X, Y, Z) nodal coordinates in ABI layout."""
    P = spec["P"]
    xi = gll.nodes(P)

    def c1(v):
        v = np.asarray(v)
        h = np.diff(v)
        return v[:-1, None] + h[:, None] * (1.0 + xi[None, :]) / 2.0

    X, Y, Z = c1(spec["xv"]), c1(spec["yv"]), c1(spec["zv"])
    nx, ny, nz, n = spec["nx"], spec["ny"], spec["nz"], P + 1
    shp = (nz, ny, nx, n, n, n)
    Xa = np.broadcast_to(X[None, None, :, None, None, :], shp).reshape(-1)
    Ya = np.broadcast_to(Y[None, :, None, None, :, None], shp).reshape(-1)
    Za = np.broadcast_to(Z[:, None, None, :, None, None], shp).reshape(-1)
    return Xa, Ya, Za


def manufactured_u(spec):
    X, Y, Z = node_coords(spec)
    return np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y) * np.sin(2 * np.pi * Z)


def channel_nu(spec, nu0=1e-3):
    """nu(x) = nu0 (1 + 0.5 sin(2 pi x) cos(2 pi y)) at the nodes."""
    X, Y, _ = node_coords(spec)
    return nu0 * (1.0 + 0.5 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y))
