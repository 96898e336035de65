"""Dense assembly of the SIP-DG Helmholtz matrix from basis-function evaluations.

Test infrastructure only (see the package docstring).

Every entry is A_ij = a(phi_j, phi_i) for the bilinear form of the viscous
(Helmholtz) and pressure (Poisson) sub-problems of Alg. 3 discretised as in
Sec. 3.3 of arXiv 2112.04167 (DG-SEM, tensor-product Lagrange polynomials on
GLL points, interior penalty):

  a(u,v) = sum_K int_K nu grad u . grad v + lambda int_K u v
         + sum_F int_F ( -{nu d_n u}[v] - {nu d_n v}[u] + sigma [u][v] ),

with all integrals by the (P+1)-point GLL rule (element and faces), [u] =
u_L - u_R and {q} = (q_L + q_R)/2 for the normal from L to R, and
sigma = max(nu_L, nu_R) (P+1)^2 / min(h_L, h_R) at each face node.  A
Dirichlet face takes [u] = u and {nu d_n u} = nu d_n u with the outward
normal and sigma = nu (P+1)^2 / h; a Neumann face adds nothing.

This construction does not use the differentiation matrix: basis values and
derivatives come from the Lagrange product formula evaluated at the
quadrature points, element by element and face by face, on full 3D arrays
(no sum factorisation).  It is meant for tiny meshes (N up to a few
thousand).
"""
import numpy as np
import scipy.linalg

from . import gll

PERIODIC, DIRICHLET, NEUMANN = 0, 1, 2


def lagrange_eval(xi, x):
    """Values V[k, j] = l_j(x_k) and derivatives dV[k, j] = l_j'(x_k) of the
    Lagrange basis on nodes xi, from the product formula."""
    xi = np.asarray(xi, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = xi.size
    V = np.ones((x.size, n))
    dV = np.zeros((x.size, n))
    for j in range(n):
        others = [m for m in range(n) if m != j]
        for k in range(x.size):
            V[k, j] = np.prod([(x[k] - xi[m]) / (xi[j] - xi[m]) for m in others])
            s = 0.0
            for q in others:
                s += (1.0 / (xi[j] - xi[q])) * np.prod(
                    [(x[k] - xi[m]) / (xi[j] - xi[m]) for m in others if m != q])
            dV[k, j] = s
    return V, dV


def abi_index(spec, e, a):
    """ABI position of node a=(a,b,c) of element e=(ex,ey,ez)."""
    nx, ny, P = spec["nx"], spec["ny"], spec["P"]
    n = P + 1
    el = (e[2] * ny + e[1]) * nx + e[0]
    return el * n ** 3 + (a[2] * n + a[1]) * n + a[0]


def element_dofs(spec, e):
    n = spec["P"] + 1
    el = (e[2] * spec["ny"] + e[1]) * spec["nx"] + e[0]
    return el * n ** 3 + np.arange(n ** 3)


def _extent(spec, d, k):
    v = (spec["xv"], spec["yv"], spec["zv"])[d]
    return float(v[k + 1] - v[k])


def _nu_nodal(spec, nu):
    N = spec["nx"] * spec["ny"] * spec["nz"] * (spec["P"] + 1) ** 3
    if np.isscalar(nu):
        return np.full(N, float(nu))
    nu = np.asarray(nu, dtype=np.float64)
    assert nu.shape == (N,)
    return nu


def assemble(spec, lam, nu=1.0):
    """Dense A (ABI ordering) for mesh ``spec`` (see synth.mesh_spec)."""
    P = spec["P"]
    n = P + 1
    ne = (spec["nx"], spec["ny"], spec["nz"])
    bc = spec["bc"]
    xi = gll.nodes(P)
    w = gll.weights(P)
    N = ne[0] * ne[1] * ne[2] * n ** 3
    nuv = _nu_nodal(spec, nu)
    A = np.zeros((N, N))

    Vq, dVq = lagrange_eval(xi, xi)          # at the volume quadrature points
    Vf, dVf = lagrange_eval(xi, [-1.0, 1.0])  # at the two ends of [-1, 1]

    # full 3D tables, index order (c, b, a) with a fastest, for points and basis
    def tensor3(Tz, Ty, Tx):
        return np.einsum("cf,be,ad->cbafed", Tz, Ty, Tx).reshape(n ** 3, n ** 3)

    Phi = tensor3(Vq, Vq, Vq)
    G = [tensor3(Vq, Vq, dVq), tensor3(Vq, dVq, Vq), tensor3(dVq, Vq, Vq)]
    Wq = np.einsum("c,b,a->cba", w, w, w).reshape(-1)

    for ez in range(ne[2]):
        for ey in range(ne[1]):
            for ex in range(ne[0]):
                e = (ex, ey, ez)
                h = [_extent(spec, d, e[d]) for d in range(3)]
                J = h[0] * h[1] * h[2] / 8.0
                dofs = element_dofs(spec, e)
                nuq = nuv[dofs]
                Ae = lam * Phi.T @ np.diag(J * Wq) @ Phi
                for d in range(3):
                    Gd = (2.0 / h[d]) * G[d]
                    Ae += Gd.T @ np.diag(J * Wq * nuq) @ Gd
                A[np.ix_(dofs, dofs)] += Ae

    # face tables: trace T[f, j] and +e_d derivative N[f, j] (reference units)
    # for the face at reference coordinate s = -1 (index 0) or +1 (index 1)
    def face_tables(d, s):
        ends = [Vf[s], dVf[s]]  # values / derivatives of the 1D basis at the end
        # face nodes (i2, i1) over the two tangential axes t1=(d+1)%3, t2=(d+2)%3
        T = np.zeros((n, n, n ** 3))
        Nd = np.zeros((n, n, n ** 3))
        t1, t2 = (d + 1) % 3, (d + 2) % 3
        for i2 in range(n):
            for i1 in range(n):
                pt = [None, None, None]
                pt[t1], pt[t2] = i1, i2
                # basis j = (ja, jb, jc); value = prod over axes
                for jc in range(n):
                    for jb in range(n):
                        for ja in range(n):
                            jj = (ja, jb, jc)
                            val, der = 1.0, 1.0
                            for ax in range(3):
                                if ax == d:
                                    val *= ends[0][jj[ax]]
                                    der *= ends[1][jj[ax]]
                                else:
                                    val *= Vq[pt[ax], jj[ax]]
                                    der *= Vq[pt[ax], jj[ax]]
                            col = (jc * n + jb) * n + ja
                            T[i2, i1, col] = val
                            Nd[i2, i1, col] = der
        return T.reshape(n * n, n ** 3), Nd.reshape(n * n, n ** 3)

    def face_node_dofs(e, d, layer):
        t1, t2 = (d + 1) % 3, (d + 2) % 3
        out = np.zeros(n * n, dtype=np.int64)
        for i2 in range(n):
            for i1 in range(n):
                a = [0, 0, 0]
                a[d], a[t1], a[t2] = layer, i1, i2
                out[i2 * n + i1] = abi_index(spec, e, a)
        return out

    for d in range(3):
        TL, NL = face_tables(d, 1)   # L side of a face: its high end
        TR, NR = face_tables(d, 0)   # R side: its low end
        t1, t2 = (d + 1) % 3, (d + 2) % 3
        for ez in range(ne[2]):
            for ey in range(ne[1]):
                for ex in range(ne[0]):
                    e = (ex, ey, ez)
                    hL = _extent(spec, d, e[d])
                    omega = np.einsum("b,a->ba", w, w).reshape(-1) * (
                        _extent(spec, t1, e[t1]) * _extent(spec, t2, e[t2]) / 4.0)
                    dofL = element_dofs(spec, e)
                    nuL = nuv[face_node_dofs(e, d, P)]
                    # high face of e
                    k = e[d] + 1
                    if k < ne[d] or bc[d] == PERIODIC:
                        r = list(e)
                        r[d] = k % ne[d]
                        r = tuple(r)
                        hR = _extent(spec, d, r[d])
                        dofR = element_dofs(spec, r)
                        nuR = nuv[face_node_dofs(r, d, 0)]
                        sigma = np.maximum(nuL, nuR) * n * n / min(hL, hR)
                        jmp = np.hstack([TL, -TR])
                        avg = 0.5 * np.hstack([nuL[:, None] * (2.0 / hL) * NL,
                                               nuR[:, None] * (2.0 / hR) * NR])
                        Af = (-jmp.T @ np.diag(omega) @ avg - avg.T @ np.diag(omega) @ jmp
                              + jmp.T @ np.diag(omega * sigma) @ jmp)
                        dofs = np.concatenate([dofL, dofR])
                        np.add.at(A, (dofs[:, None], dofs[None, :]), Af)
                    elif bc[d] == DIRICHLET:
                        sigma = nuL * n * n / hL
                        jmp = TL
                        avg = nuL[:, None] * (2.0 / hL) * NL   # outward normal = +e_d
                        Af = (-jmp.T @ np.diag(omega) @ avg - avg.T @ np.diag(omega) @ jmp
                              + jmp.T @ np.diag(omega * sigma) @ jmp)
                        A[np.ix_(dofL, dofL)] += Af
                    # low boundary face of e
                    if e[d] == 0 and bc[d] == DIRICHLET:
                        nu0 = nuv[face_node_dofs(e, d, 0)]
                        sigma = nu0 * n * n / hL
                        jmp = TR
                        avg = -nu0[:, None] * (2.0 / hL) * NR  # outward normal = -e_d
                        Af = (-jmp.T @ np.diag(omega) @ avg - avg.T @ np.diag(omega) @ jmp
                              + jmp.T @ np.diag(omega * sigma) @ jmp)
                        A[np.ix_(dofL, dofL)] += Af
    return A


def dirichlet_load(spec, nu, g):
    """Load vector of inhomogeneous Dirichlet data (Nitsche terms of the SIP
    form): for every node i, sum over the Dirichlet faces F of
        int_F sigma g phi_i - int_F nu d_n(phi_i) g,
    sigma = nu (P+1)^2 / h as in the bilinear form, n the outward normal, all
    face integrals by the GLL rule.  g: nodal field (ABI layout) whose values
    at the Dirichlet face nodes are the data; nu: scalar or nodal field.
    A x = M f + dirichlet_load(spec, nu, g) is the SIP problem with u = g on
    the Dirichlet faces."""
    P = spec["P"]
    n = P + 1
    ne = (spec["nx"], spec["ny"], spec["nz"])
    xi = gll.nodes(P)
    w = gll.weights(P)
    nuv = _nu_nodal(spec, nu)
    g = np.asarray(g, dtype=np.float64)
    _, dVf = lagrange_eval(xi, [-1.0, 1.0])   # dVf[s, j] = l_j'(+-1)
    L = np.zeros(g.size)
    for d in range(3):
        if spec["bc"][d] != DIRICHLET:
            continue
        t1, t2 = [k for k in range(3) if k != d]
        for ez in range(ne[2]):
            for ey in range(ne[1]):
                for ex in range(ne[0]):
                    e = (ex, ey, ez)
                    for high in (False, True):
                        if e[d] != (ne[d] - 1 if high else 0):
                            continue
                        h = _extent(spec, d, e[d])
                        om_t = _extent(spec, t1, e[t1]) * _extent(spec, t2, e[t2]) / 4.0
                        layer = P if high else 0
                        sgn = 1.0 if high else -1.0
                        for i2 in range(n):
                            for i1 in range(n):
                                a = [0, 0, 0]
                                a[d], a[t1], a[t2] = layer, i1, i2
                                f = abi_index(spec, e, a)
                                om = w[i1] * w[i2] * om_t
                                sigma = nuv[f] * n * n / h
                                L[f] += om * sigma * g[f]
                                for k in range(n):      # the normal line through the face node
                                    a[d] = k
                                    j = abi_index(spec, e, a)
                                    dn = sgn * (2.0 / h) * dVf[1 if high else 0, k]
                                    L[j] -= om * nuv[f] * dn * g[f]
    return L


def mass_diag(spec):
    """Diagonal GLL mass matrix J w_a w_b w_c in ABI layout."""
    P = spec["P"]
    n = P + 1
    w = gll.weights(P)
    hx = np.diff(spec["xv"])
    hy = np.diff(spec["yv"])
    hz = np.diff(spec["zv"])
    Jel = np.einsum("k,j,i->kji", hz, hy, hx) / 8.0          # (ez, ey, ex)
    W = np.einsum("c,b,a->cba", w, w, w)
    return np.einsum("kji,cba->kjicba", Jel, W).reshape(-1)


def singular(spec, lam):
    """True when lambda = 0 and no Dirichlet face exists (constants in the kernel)."""
    return lam == 0.0 and all(b != DIRICHLET for b in spec["bc"])


def solve(spec, A, b, lam):
    """Exact discrete solution of A x = b: Cholesky, or for the singular
    problem the bordered system fixing sum(M x) = 0 after projecting b to mean
    zero."""
    if not singular(spec, lam):
        c = scipy.linalg.cho_factor(A)
        return scipy.linalg.cho_solve(c, b)
    N = A.shape[0]
    m = mass_diag(spec)
    bb = b - b.mean()
    K = np.zeros((N + 1, N + 1))
    K[:N, :N] = A
    K[:N, N] = m
    K[N, :N] = m
    sol = scipy.linalg.solve(K, np.concatenate([bb, [0.0]]))
    return sol[:N]
