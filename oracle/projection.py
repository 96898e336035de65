"""DG divergence, gradient and the projection substep with a pressure of
degree P-1 (oracle).

Test infrastructure only (see the package docstring).

Alg. 3 of arXiv 2112.04167 corrects the predicted velocity v' by

    solve  lap(psi) = div v',   d_n psi = n.(v' - v_b) on the boundary,
    v'' = v' - grad psi,

and Sec. 3.3 puts the velocity at degree P and the pressure at degree P-1
(tensor-product Lagrange polynomials on GLL points, DG-SEM, interior penalty
for the pressure problem).  The paper gives no DG formulas for these
operators; the reading used here (written out in the build's design notes):

  * weak divergence with a central flux, against every pressure basis
    function q (degree P-1):
        D(v; v_b)_q = - sum_K int_K v . grad q
                      + sum_F(interior) int_F {v}.n [q]
                      + sum_F(boundary) int_F (v_b . n_out) q
    (for smooth v this is int (div v) q, with v . n taken from v_b on the
    boundary);
  * the pressure problem in weak form with the Neumann data folded in:
        a_SIP(psi, q) = -D(v'; v_b)_q   for all q,
    since int grad psi . grad q = int v'.grad q - int_boundary (v_b.n) q
    once d_n psi = n.(v' - v_b) is substituted; a_SIP is the SIP form of
    degree P-1 with natural (Neumann) boundaries, which is singular: the load
    is projected to mean zero and psi returned with M-weighted mean zero
    (as for the pressure Poisson problem of the hot path);
  * the gradient is the negative adjoint of D without boundary data under the
    GLL masses, (G psi, w)_{M_v} = -(psi, D(w; 0)):
        (G psi, w) = sum_K int_K grad psi . w - sum_F(interior) int_F [psi] n.{w},
    i.e. at velocity nodes: the derivative of the P-1 interpolant, minus the
    jump of psi across each interior face lifted onto that face's nodes;
  * every integral by the (P+1)-point GLL rule of the velocity, which is
    exact here (degree 2P-1 per direction).

These functions evaluate the basis functions element by element and face by
face on full 3D arrays (no sum factorisation); tiny and small meshes only.
"""
import numpy as np

from . import dense, gll, kron

PERIODIC, DIRICHLET, NEUMANN = 0, 1, 2


def pressure_spec(spec):
    """The same mesh at degree P-1 with the pressure BCs (Dirichlet axes
    become Neumann axes)."""
    p = dict(spec)
    p["P"] = spec["P"] - 1
    p["bc"] = tuple(NEUMANN if b == DIRICHLET else b for b in spec["bc"])
    return p


def _tables(P, Q):
    """Velocity GLL nodes/weights (degree P) and the Lagrange basis of the
    scalar space (degree Q: P-1 for the pressure, P for the equal-order
    operators of the variable-viscosity terms) with its derivative at the
    velocity nodes: Vq[a, i], dVq[a, i]."""
    xv, wv = gll.nodes(P), gll.weights(P)
    xp = gll.nodes(Q)
    Vq, dVq = dense.lagrange_eval(xp, xv)
    return xv, wv, Vq, dVq


def _extents(spec):
    return [np.diff(np.asarray(spec[k], dtype=np.float64)) for k in ("xv", "yv", "zv")]


def _elements(spec):
    for ez in range(spec["nz"]):
        for ey in range(spec["ny"]):
            for ex in range(spec["nx"]):
                yield (ex, ey, ez), (ez * spec["ny"] + ey) * spec["nx"] + ex


def divergence(spec, v, vb=None, q_degree=None):
    """Weak divergence D(v; v_b) on the pressure basis (ABI layout of the
    degree P-1 mesh; q_degree = P: on the velocity basis itself).  v, vb:
    three nodal arrays (ABI layout, degree P); vb None means v_b = 0."""
    P = spec["P"]
    Q = P - 1 if q_degree is None else q_degree
    n, m = P + 1, Q + 1
    xv, wv, Vq, dVq = _tables(P, Q)
    h = _extents(spec)
    nn = (spec["nx"], spec["ny"], spec["nz"])
    nel = nn[0] * nn[1] * nn[2]
    V = [np.asarray(c, dtype=np.float64).reshape(nel, n, n, n) for c in v]   # [el][c][b][a]
    Vb = None if vb is None else [np.asarray(c, dtype=np.float64).reshape(nel, n, n, n) for c in vb]
    out = np.zeros((nel, m, m, m))                                           # [el][iz][iy][ix]
    W = np.einsum("c,b,a->cba", wv, wv, wv)
    # basis factors per direction at the velocity nodes: value / derivative
    for e, el in _elements(spec):
        hx, hy, hz = h[0][e[0]], h[1][e[1]], h[2][e[2]]
        J = hx * hy * hz / 8.0
        for d, hd in enumerate((hx, hy, hz)):
            t = W * J * V[d][el]                                              # [c][b][a]
            A = [Vq, Vq, Vq]
            A[d] = dVq * (2.0 / hd)
            # out[iz,iy,ix] -= sum_{c,b,a} Az[c,iz] Ay[b,iy] Ax[a,ix] t[c,b,a]
            out[el] -= np.einsum("cz,by,ax,cba->zyx", A[2], A[1], A[0], t)
    # faces
    for d in range(3):
        for e, el in _elements(spec):
            hs = [h[k][e[k]] for k in range(3)]
            t1, t2 = [k for k in range(3) if k != d]
            omega = np.outer(wv, wv) * hs[t1] * hs[t2] / 4.0                 # [node t2][node t1]
            for high in (False, True):
                nb = list(e)
                nb[d] += 1 if high else -1
                inside = 0 <= nb[d] < nn[d]
                if not inside and spec["bc"][d] == PERIODIC:
                    nb[d] %= nn[d]
                    inside = True
                layer = n - 1 if high else 0
                if inside:
                    elnb = (nb[2] * nn[1] + nb[1]) * nn[0] + nb[0]
                    own = _face(V[d][el], d, layer)
                    oth = _face(V[d][elnb], d, 0 if high else n - 1)
                    f = 0.5 * (own + oth)
                elif Vb is not None:
                    f = _face(Vb[d][el], d, layer)
                else:
                    continue
                sgn = 1.0 if high else -1.0   # [q] = q_L - q_R with n from L to R; boundary: n_out
                g = sgn * omega * f                                           # [t2 node][t1 node]
                val = np.einsum("ts,sy,tz->zy", g, Vq, Vq)                    # [i_t2][i_t1]
                ip = m - 1 if high else 0
                _add_face(out[el], d, ip, val)
    return out.reshape(-1)


def _face(arr, d, layer):
    """Face layer of an element array [c][b][a] normal to axis d, indexed
    [t2][t1] with t1 < t2 the tangential axes."""
    if d == 0:
        return arr[:, :, layer]          # [c][b]
    if d == 1:
        return arr[:, layer, :]          # [c][a]
    return arr[layer, :, :]              # [b][a]


def _add_face(arr, d, layer, val):
    if d == 0:
        arr[:, :, layer] += val
    elif d == 1:
        arr[:, layer, :] += val
    else:
        arr[layer, :, :] += val


def gradient(spec, psi, q_degree=None):
    """Nodal gradient G psi on the velocity nodes: three arrays (ABI layout,
    degree P), psi in the ABI layout of the degree P-1 mesh (q_degree = P:
    of the velocity mesh itself)."""
    P = spec["P"]
    Q = P - 1 if q_degree is None else q_degree
    n, m = P + 1, Q + 1
    xv, wv, Vq, dVq = _tables(P, Q)
    h = _extents(spec)
    nn = (spec["nx"], spec["ny"], spec["nz"])
    nel = nn[0] * nn[1] * nn[2]
    Q = np.asarray(psi, dtype=np.float64).reshape(nel, m, m, m)              # [el][iz][iy][ix]
    G = [np.zeros((nel, n, n, n)) for _ in range(3)]
    for e, el in _elements(spec):
        hs = (h[0][e[0]], h[1][e[1]], h[2][e[2]])
        for d in range(3):
            A = [Vq, Vq, Vq]
            A[d] = dVq * (2.0 / hs[d])
            G[d][el] += np.einsum("cz,by,ax,zyx->cba", A[2], A[1], A[0], Q[el])
    # face terms: -[psi] n.{w} lifted onto the face nodes, divided by the mass
    for d in range(3):
        for e, el in _elements(spec):
            nb = list(e)
            nb[d] += 1
            if nb[d] >= nn[d]:
                if spec["bc"][d] != PERIODIC:
                    continue
                nb[d] = 0
            elnb = (nb[2] * nn[1] + nb[1]) * nn[0] + nb[0]
            # pressure traces on the velocity face nodes
            trL = _ptrace(Q[el], d, m - 1, Vq)
            trR = _ptrace(Q[elnb], d, 0, Vq)
            jump = trL - trR                                                  # [t2 node][t1 node]
            hL, hR = h[d][e[d]], h[d][nb[d]]
            # int_F {w}[psi] / M at the node: (1/2) w_t1 w_t2 h_t1 h_t2 / 4 over
            # w_P w_t1 w_t2 h_d h_t1 h_t2 / 8 = 1 / (w_P h_d)
            _add_face(G[d][el], d, n - 1, -jump / (wv[-1] * hL))
            _add_face(G[d][elnb], d, 0, -jump / (wv[0] * hR))
    return [g.reshape(-1) for g in G]


def _ptrace(Qe, d, layer, Vq):
    """Pressure element [iz][iy][ix] restricted to its face layer normal to d,
    interpolated to the velocity face nodes: [t2 node][t1 node]."""
    if d == 0:
        f = Qe[:, :, layer]                 # [iz][iy]
    elif d == 1:
        f = Qe[:, layer, :]                 # [iz][ix]
    else:
        f = Qe[layer, :, :]                 # [iy][ix]
    return Vq @ f @ Vq.T                    # [node t2][node t1]


def project(spec, v, vb=None):
    """The projection substep: psi from a_SIP(psi, q) = -D(v; v_b)_q on the
    degree P-1 mesh (natural boundaries, singular: load projected, psi with
    M-weighted mean zero), then v'' = v - G psi.  Returns (v'', psi)."""
    ps = pressure_spec(spec)
    rhs = -divergence(spec, v, vb)
    psi = kron.FDM(ps, 0.0).solve(rhs)
    g = gradient(spec, psi)
    return [np.asarray(v[d], dtype=np.float64) - g[d] for d in range(3)], psi
