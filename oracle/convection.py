"""Convective term F_c = -div(v v) with local Lax-Friedrichs fluxes, and the
viscous term F_d2 = div(nu (grad v)^T) (oracle).

Test infrastructure only (see the package docstring).

Sec. 3.3 of arXiv 2112.04167 discretises convection by DG-SEM with
consistent integration and local Lax-Friedrichs fluxes; the paper gives no
formulas beyond that.  The reading used here (written out in the build's
design notes):

  * weak form per component i, test functions phi of the velocity basis
    (degree P on GLL nodes), outward normal n of element K:
        (M F_c,i)_phi = sum_K int_K sum_k v_k v_i d_k phi
                        - sum_K int_dK H_i phi,
        H_i = ( (v-.n) v-_i + (v+.n) v+_i ) / 2 + alpha (v-_i - v+_i) / 2,
        alpha = 2 max(|v-.n|, |v+.n|),
    v- the element's own trace, v+ the neighbour's (periodic axes wrap) or,
    on a wall, the boundary state v_b (zero when not given); alpha is the
    spectral radius of the Jacobian of u -> (u.n) u, taken pointwise;
  * "consistent integration": every integral by the Gauss-Legendre rule with
    Q = floor(3P/2) + 1 points per direction, exact for the polynomial part
    (degree 3P per direction); M is the GLL (collocation) mass of the
    velocity, as in every other term;
  * F_d2,i = sum_k d_k (nu d_i v_k): the equal-order DG gradient G of each
    component v_k (its i-th component is d_i v_k), times nu at the nodes,
    then the equal-order weak divergence D of the vector field
    (nu d_i v_0, nu d_i v_1, nu d_i v_2) with that field's own trace as the
    boundary data, divided by the GLL mass.

Full 3D arrays element by element and face by face (no sum factorisation);
tiny and small meshes only.
"""
import numpy as np

from . import dense, gll, projection

PERIODIC = 0


def quad_points(P):
    """Gauss-Legendre points per direction for the convective integrals."""
    return 3 * P // 2 + 1


def _tables(P):
    Q = quad_points(P)
    xg, wg = np.polynomial.legendre.leggauss(Q)
    B, dB = dense.lagrange_eval(gll.nodes(P), xg)   # B[q, a] = l_a(x_q)
    return xg, wg, B, dB


def _face_layer(arr, d, layer):
    """[t2][t1] face layer of an element array [c][b][a] normal to axis d."""
    if d == 0:
        return arr[:, :, layer]
    if d == 1:
        return arr[:, layer, :]
    return arr[layer, :, :]


def _add_face(arr, d, layer, val):
    if d == 0:
        arr[:, :, layer] += val
    elif d == 1:
        arr[:, layer, :] += val
    else:
        arr[layer, :, :] += val


def convection(spec, v, vb=None):
    """F_c = -div(v v) as three nodal fields (ABI layout, degree P)."""
    P = spec["P"]
    n = P + 1
    _, wg, B, dB = _tables(P)
    h = [np.diff(np.asarray(spec[k], dtype=np.float64)) for k in ("xv", "yv", "zv")]
    nn = (spec["nx"], spec["ny"], spec["nz"])
    nel = nn[0] * nn[1] * nn[2]
    V = [np.asarray(c, dtype=np.float64).reshape(nel, n, n, n) for c in v]
    Vb = None if vb is None else [np.asarray(c, dtype=np.float64).reshape(nel, n, n, n) for c in vb]
    out = [np.zeros((nel, n, n, n)) for _ in range(3)]
    W = np.einsum("z,y,x->zyx", wg, wg, wg)

    def elements():
        for ez in range(nn[2]):
            for ey in range(nn[1]):
                for ex in range(nn[0]):
                    yield (ex, ey, ez), (ez * nn[1] + ey) * nn[0] + ex

    # volume: int_K v_k v_i d_k phi at the Gauss points
    for e, el in elements():
        hs = [h[k][e[k]] for k in range(3)]
        J = hs[0] * hs[1] * hs[2] / 8.0
        U = [np.einsum("zc,yb,xa,cba->zyx", B, B, B, V[k][el]) for k in range(3)]
        for i in range(3):
            for k in range(3):
                F = W * J * U[i] * U[k]
                T = [B, B, B]
                T[k] = dB * (2.0 / hs[k])
                out[i][el] += np.einsum("zc,yb,xa,zyx->cba", T[2], T[1], T[0], F)
    # faces: - int_dK H_i phi, each element over its own six faces
    for e, el in elements():
        hs = [h[k][e[k]] for k in range(3)]
        for d in range(3):
            t1, t2 = [k for k in range(3) if k != d]
            omega = np.outer(wg, wg) * hs[t1] * hs[t2] / 4.0          # [q t2][q t1]
            for high in (False, True):
                layer = n - 1 if high else 0
                nb = list(e)
                nb[d] += 1 if high else -1
                inside = 0 <= nb[d] < nn[d]
                if not inside and spec["bc"][d] == PERIODIC:
                    nb[d] %= nn[d]
                    inside = True
                own = [B @ _face_layer(V[k][el], d, layer) @ B.T for k in range(3)]
                if inside:
                    elnb = (nb[2] * nn[1] + nb[1]) * nn[0] + nb[0]
                    oth = [B @ _face_layer(V[k][elnb], d, 0 if high else n - 1) @ B.T for k in range(3)]
                elif Vb is not None:
                    oth = [B @ _face_layer(Vb[k][el], d, layer) @ B.T for k in range(3)]
                else:
                    oth = [np.zeros_like(own[0]) for _ in range(3)]
                sgn = 1.0 if high else -1.0
                vnm, vnp = sgn * own[d], sgn * oth[d]
                alpha = 2.0 * np.maximum(np.abs(vnm), np.abs(vnp))
                for i in range(3):
                    H = 0.5 * (vnm * own[i] + vnp * oth[i]) + 0.5 * alpha * (own[i] - oth[i])
                    _add_face(out[i][el], d, layer, -(B.T @ (omega * H) @ B))
    M = dense.mass_diag(spec)
    return [o.reshape(-1) / M for o in out]


def fd2(spec, nu, v):
    """F_d2 = div(nu (grad v)^T) as three nodal fields (equal-order DG
    gradient and divergence)."""
    P = spec["P"]
    M = dense.mass_diag(spec)
    nu = np.asarray(nu, dtype=np.float64)
    grads = [projection.gradient(spec, np.asarray(c, dtype=np.float64), q_degree=P) for c in v]  # grads[k][i] = d_i v_k
    out = []
    for i in range(3):
        w = [nu * grads[k][i] for k in range(3)]
        out.append(projection.divergence(spec, w, w, q_degree=P) / M)
    return out
