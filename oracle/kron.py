"""1D SIP-DG matrices, Kronecker-sum assembly and the fast-diagonalisation
exact solver (oracle).

Test infrastructure only (see the package docstring).

On a Cartesian product grid with constant nu and GLL-collocated quadrature
(Sec. 3.3 of arXiv 2112.04167: DG-SEM on tensor-product GLL hexahedra,
interior penalty), every volume and face integral of the Helmholtz form
factorises into a 1D term times the 1D GLL masses of the other two axes, so
in global tensor ordering (x fastest, global 1D index = e*(P+1) + a)

    A = lambda Mz(x)My(x)Mx + Mz(x)My(x)Kx + Mz(x)Ky(x)Mx + Kz(x)My(x)Mx,

with M_d = diag(h/2 w) and K_d the 1D SIP matrix of that axis (same penalty
rule sigma = nu (P+1)^2 / min(h_L, h_R), same BC).  The exact discrete
solution then follows from the generalized eigenproblems K_d S = M_d S Lam,
S^T M_d S = I (fast diagonalisation, Lynch, Rice & Thomas 1964):

    x* = (Sz(x)Sy(x)Sx) (lambda + Lx (+) Ly (+) Lz)^-1 (Sz(x)Sy(x)Sx)^T b.

For the singular Poisson problem (lambda = 0, no Dirichlet axis) the load is
projected to Euclidean mean zero first and the zero mode is dropped, which
returns the solution with M-weighted mean zero.
"""
import numpy as np
import scipy.linalg

from . import gll

PERIODIC, DIRICHLET, NEUMANN = 0, 1, 2


def sip_1d(v, P, bc, nu=1.0):
    """(K, Mdiag) of the 1D SIP operator on vertices v with degree P."""
    v = np.asarray(v, dtype=np.float64)
    ne = v.size - 1
    n = P + 1
    w = gll.weights(P)
    D = gll.diff_matrix(P)
    N1 = ne * n
    K = np.zeros((N1, N1))
    M = np.zeros(N1)
    h = np.diff(v)
    for e in range(ne):
        s = slice(e * n, (e + 1) * n)
        g = 2.0 / h[e]
        M[s] = 0.5 * h[e] * w
        K[s, s] += nu * (0.5 * h[e]) * g * g * (D.T @ np.diag(w) @ D)

    def add(dofs, jmp, avg, sigma):
        Kf = -np.outer(jmp, avg) - np.outer(avg, jmp) + sigma * np.outer(jmp, jmp)
        np.add.at(K, (dofs[:, None], dofs[None, :]), Kf)

    eP = np.zeros(n)
    eP[-1] = 1.0
    e0 = np.zeros(n)
    e0[0] = 1.0
    for e in range(ne):
        dL = np.arange(e * n, (e + 1) * n)
        if e + 1 < ne or bc == PERIODIC:
            r = (e + 1) % ne
            dR = np.arange(r * n, (r + 1) * n)
            sigma = nu * n * n / min(h[e], h[r])
            jmp = np.concatenate([eP, -e0])
            avg = 0.5 * nu * np.concatenate([(2.0 / h[e]) * D[P, :], (2.0 / h[r]) * D[0, :]])
            add(np.concatenate([dL, dR]), jmp, avg, sigma)
        elif bc == DIRICHLET:
            add(dL, eP, nu * (2.0 / h[e]) * D[P, :], nu * n * n / h[e])
    if bc == DIRICHLET:
        add(np.arange(n), e0, -nu * (2.0 / h[0]) * D[0, :], nu * n * n / h[0])
    return K, M


def axes(spec, nu=1.0):
    """[(K_x, M_x), (K_y, M_y), (K_z, M_z)]."""
    P = spec["P"]
    return [sip_1d(spec[k], P, spec["bc"][d], nu) for d, k in enumerate(("xv", "yv", "zv"))]


def abi_to_global(spec, u):
    """ABI layout -> global tensor (Z, Y, X) with X = ex*(P+1)+a."""
    n = spec["P"] + 1
    nx, ny, nz = spec["nx"], spec["ny"], spec["nz"]
    t = np.asarray(u).reshape(nz, ny, nx, n, n, n)          # ez ey ex c b a
    return t.transpose(0, 3, 1, 4, 2, 5).reshape(nz * n, ny * n, nx * n)


def global_to_abi(spec, U):
    n = spec["P"] + 1
    nx, ny, nz = spec["nx"], spec["ny"], spec["nz"]
    t = np.asarray(U).reshape(nz, n, ny, n, nx, n)           # ez c ey b ex a
    return t.transpose(0, 2, 4, 1, 3, 5).reshape(-1)


def assemble(spec, lam, nu=1.0):
    """Dense A by the Kronecker sum, returned in ABI ordering (tiny meshes)."""
    (Kx, Mx), (Ky, My), (Kz, Mz) = axes(spec, nu)
    Mx, My, Mz = np.diag(Mx), np.diag(My), np.diag(Mz)
    A = (lam * np.kron(Mz, np.kron(My, Mx)) + np.kron(Mz, np.kron(My, Kx))
         + np.kron(Mz, np.kron(Ky, Mx)) + np.kron(Kz, np.kron(My, Mx)))
    N = A.shape[0]
    perm = global_to_abi(spec, np.arange(N))   # perm[abi] = global index
    return A[np.ix_(perm, perm)]


class FDM:
    """Fast-diagonalisation exact solver for constant nu."""

    def __init__(self, spec, lam, nu=1.0):
        self.spec, self.lam, self.nu = spec, float(lam), float(nu)
        self.S, self.L, self.M = [], [], []
        for K, M in axes(spec, nu):
            L, S = scipy.linalg.eigh(K, np.diag(M))
            self.S.append(S)
            self.L.append(L)
            self.M.append(M)
        Lx, Ly, Lz = self.L
        self.den = lam + Lz[:, None, None] + Ly[None, :, None] + Lx[None, None, :]
        self.singular = lam == 0.0 and all(b != DIRICHLET for b in spec["bc"])
        if self.singular:
            # the zero mode of each periodic/Neumann axis is its smallest eigenvalue
            self.den[0, 0, 0] = np.inf

    @staticmethod
    def _apply_tensor(U, Ax, Ay, Az):
        """out[k,j,i] = sum_{z,y,x} Az[k,z] Ay[j,y] Ax[i,x] U[z,y,x]."""
        U = U @ Ax.T
        U = np.matmul(Ay, U)
        Z = U.shape[0]
        return (Az @ U.reshape(Z, -1)).reshape(Az.shape[0], U.shape[1], U.shape[2])

    def solve(self, b):
        """x* for the load vector b (ABI layout)."""
        b = np.asarray(b, dtype=np.float64)
        if self.singular:
            b = b - b.mean()
        B = abi_to_global(self.spec, b)
        Sx, Sy, Sz = self.S
        Bh = self._apply_tensor(B, Sx.T, Sy.T, Sz.T)
        X = self._apply_tensor(Bh / self.den, Sx, Sy, Sz)
        x = global_to_abi(self.spec, X)
        if self.singular:
            m = np.einsum("k,j,i->kji", self.M[2], self.M[1], self.M[0])
            m = global_to_abi(self.spec, m)
            x = x - np.dot(m, x) / m.sum()
        return x

    def apply_inverse(self, r):
        """(Sz(x)Sy(x)Sx) (lambda + Lx(+)Ly(+)Lz)^-1 (Sz(x)Sy(x)Sx)^T r, the
        zero mode dropped when singular, with no projection or shift: the
        fast-diagonalisation preconditioner as defined (ABI layout in and out)."""
        R = abi_to_global(self.spec, np.asarray(r, dtype=np.float64))
        Sx, Sy, Sz = self.S
        T = self._apply_tensor(R, Sx.T, Sy.T, Sz.T) / self.den
        return global_to_abi(self.spec, self._apply_tensor(T, Sx, Sy, Sz))

    def eigenvalues_generalized(self):
        """Spectrum of M^-1 A: lambda + Lx(+)Ly(+)Lz (zero mode excluded if singular)."""
        ev = self.den.reshape(-1)
        return np.sort(ev[np.isfinite(ev)])
