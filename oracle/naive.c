/*
 * Oracle: naive matrix-free SIP-DG Helmholtz apply and Jacobi diagonal, FP64.
 *
 * TEST INFRASTRUCTURE ONLY -- linked by nothing in the product library; used
 * by the tests, the smoke check and the CPU-baseline leg of the benchmark.
 *
 * Operator (arXiv 2112.04167, Sec. 3.3: DG-SEM on tensor-product GLL
 * hexahedra, interior penalty for the viscous and pressure problems; Alg. 3:
 * the implicit sub-problems lambda u - div(nu grad u) = f).  With GLL
 * collocated quadrature everywhere, y = A x is
 *
 *   a(u,v) = sum_K int_K (nu grad u . grad v + lambda u v)
 *          + sum_F int_F ( -{nu d_n u}[v] - {nu d_n v}[u] + sigma [u][v] )
 *
 * [u] = u_L - u_R, {q} = (q_L + q_R)/2 with the normal n from L to R;
 * sigma = max(nu_L, nu_R) (P+1)^2 / min(h_L, h_R) (h = extent normal to F).
 * On a Dirichlet face [u] = u, {nu d_n u} = nu d_n u (outward normal),
 * sigma = nu (P+1)^2 / h.  Neumann faces contribute nothing; periodic axes
 * wrap around.
 *
 * Data layout: node (a,b,c) of element (ex,ey,ez) is stored at
 *   ((ez*ny + ey)*nx + ex)*(P+1)^3 + (c*(P+1) + b)*(P+1) + a,
 * element extents come from the vertex arrays xv[nx+1], yv[ny+1], zv[nz+1].
 *
 * The element loop is the plain one: every element gathers its own row block,
 * recomputing the neighbour traces and normal derivatives it needs.  OpenMP
 * uses a static schedule; every output entry is computed by exactly one
 * thread in a fixed order, so results do not depend on the thread count.
 */
#include <math.h>
#include <stddef.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXN 16

typedef struct {
    int n[3];          /* elements per axis */
    int P, np;         /* degree, nodes per direction */
    const double *v[3];/* vertex arrays */
    const int *bc;     /* per-axis BC: 0 periodic, 1 Dirichlet, 2 Neumann */
    const double *D, *w;
} mesh_t;

static inline size_t node_index(const mesh_t *m, const int e[3], const int a[3])
{
    const size_t np = (size_t)m->np;
    size_t el = ((size_t)e[2] * m->n[1] + e[1]) * m->n[0] + e[0];
    return el * np * np * np + ((size_t)a[2] * np + a[1]) * np + a[0];
}

static inline double extent(const mesh_t *m, int d, int k) { return m->v[d][k + 1] - m->v[d][k]; }

/* neighbour element index along axis d in direction s (-1 / +1); returns 0 if
   the face is on the domain boundary of a non-periodic axis. */
static int neighbour(const mesh_t *m, const int e[3], int d, int s, int nb[3])
{
    nb[0] = e[0]; nb[1] = e[1]; nb[2] = e[2];
    int k = e[d] + s;
    if (k < 0 || k >= m->n[d]) {
        if (m->bc[d] != 0) return 0;
        k = (k + m->n[d]) % m->n[d];
    }
    nb[d] = k;
    return 1;
}

static inline double nu_at(const double *nu, double nu_const, size_t i) { return nu ? nu[i] : nu_const; }

/* one element's rows of y = A x */
static void element_apply(const mesh_t *m, const int e[3], double lambda, const double *nu,
                          double nu_const, const double *x, double *y)
{
    const int np = m->np, P = m->P;
    const double *D = m->D, *w = m->w;
    double h[3], g[3];
    for (int d = 0; d < 3; ++d) { h[d] = extent(m, d, e[d]); g[d] = 2.0 / h[d]; }
    const double J = h[0] * h[1] * h[2] / 8.0;
    double yl[MAXN * MAXN * MAXN];
    double t[MAXN * MAXN * MAXN];
    const int nloc = np * np * np;
    int a[3];

    /* mass: lambda J w_a w_b w_c x */
    for (a[2] = 0; a[2] < np; ++a[2])
        for (a[1] = 0; a[1] < np; ++a[1])
            for (a[0] = 0; a[0] < np; ++a[0]) {
                int l = (a[2] * np + a[1]) * np + a[0];
                yl[l] = lambda * J * w[a[0]] * w[a[1]] * w[a[2]] * x[node_index(m, e, a)];
            }

    /* volume: sum_d D_d^T [ J g_d^2 W nu (D_d x) ] */
    for (int d = 0; d < 3; ++d) {
        for (a[2] = 0; a[2] < np; ++a[2])
            for (a[1] = 0; a[1] < np; ++a[1])
                for (a[0] = 0; a[0] < np; ++a[0]) {
                    int q = a[d];
                    int b[3] = {a[0], a[1], a[2]};
                    double s = 0.0;
                    for (int j = 0; j < np; ++j) {
                        b[d] = j;
                        s += D[q * np + j] * x[node_index(m, e, b)];
                    }
                    size_t gi = node_index(m, e, a);
                    double W = w[a[0]] * w[a[1]] * w[a[2]];
                    t[(a[2] * np + a[1]) * np + a[0]] = J * g[d] * g[d] * W * nu_at(nu, nu_const, gi) * s;
                }
        for (a[2] = 0; a[2] < np; ++a[2])
            for (a[1] = 0; a[1] < np; ++a[1])
                for (a[0] = 0; a[0] < np; ++a[0]) {
                    int i = a[d];
                    int b[3] = {a[0], a[1], a[2]};
                    double s = 0.0;
                    for (int q = 0; q < np; ++q) {
                        b[d] = q;
                        s += D[q * np + i] * t[(b[2] * np + b[1]) * np + b[0]];
                    }
                    yl[(a[2] * np + a[1]) * np + a[0]] += s;
                }
    }

    /* faces: for every axis d and side s, the part of the face integral that
       lands in this element's rows */
    for (int d = 0; d < 3; ++d) {
        const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
        for (int s = -1; s <= 1; s += 2) {
            int nb[3];
            int interior = neighbour(m, e, d, s, nb);
            if (!interior && m->bc[d] != 1) continue; /* Neumann: natural */
            const int aown = (s > 0) ? P : 0;  /* own face layer */
            const int anb = (s > 0) ? 0 : P;   /* neighbour face layer */
            const double hnb = interior ? extent(m, d, nb[d]) : 0.0;
            for (int i2 = 0; i2 < np; ++i2)
                for (int i1 = 0; i1 < np; ++i1) {
                    const double omega = w[i1] * w[i2] * h[t1] * h[t2] / 4.0;
                    int ao[3], an[3];
                    ao[t1] = i1; ao[t2] = i2; ao[d] = aown;
                    an[t1] = i1; an[t2] = i2; an[d] = anb;
                    /* own trace and normal (+e_d) derivative */
                    double uo = x[node_index(m, e, ao)];
                    double dO = 0.0;
                    {
                        int b[3] = {ao[0], ao[1], ao[2]};
                        for (int j = 0; j < np; ++j) { b[d] = j; dO += D[aown * np + j] * x[node_index(m, e, b)]; }
                        dO *= g[d];
                    }
                    const double nuo = nu_at(nu, nu_const, node_index(m, e, ao));
                    double yface = 0.0;  /* goes to the own face node */
                    double cline = 0.0;  /* coefficient of D[aown][j] on the own line */
                    if (interior) {
                        double un = x[node_index(m, nb, an)];
                        double dN = 0.0;
                        {
                            int b[3] = {an[0], an[1], an[2]};
                            for (int j = 0; j < np; ++j) { b[d] = j; dN += D[anb * np + j] * x[node_index(m, nb, b)]; }
                            dN *= 2.0 / hnb;
                        }
                        const double nun = nu_at(nu, nu_const, node_index(m, nb, an));
                        const double sigma = fmax(nuo, nun) * np * np / fmin(h[d], hnb);
                        if (s > 0) { /* own = L, neighbour = R */
                            double jump = uo - un, avg = 0.5 * (nuo * dO + nun * dN);
                            yface = omega * (-avg + sigma * jump);
                            cline = -0.5 * omega * nuo * g[d] * jump;
                        } else {     /* neighbour = L, own = R */
                            double jump = un - uo, avg = 0.5 * (nun * dN + nuo * dO);
                            yface = omega * (avg - sigma * jump);
                            cline = -0.5 * omega * nuo * g[d] * jump;
                        }
                    } else {         /* Dirichlet (homogeneous) */
                        const double sigma = nuo * np * np / h[d];
                        if (s > 0) {
                            yface = omega * (-nuo * dO + sigma * uo);
                            cline = -omega * nuo * g[d] * uo;
                        } else {
                            yface = omega * (nuo * dO + sigma * uo);
                            cline = omega * nuo * g[d] * uo;
                        }
                    }
                    yl[(ao[2] * np + ao[1]) * np + ao[0]] += yface;
                    int b[3] = {ao[0], ao[1], ao[2]};
                    for (int j = 0; j < np; ++j) {
                        b[d] = j;
                        yl[(b[2] * np + b[1]) * np + b[0]] += cline * D[aown * np + j];
                    }
                }
        }
    }
    const size_t base = node_index(m, e, (int[3]){0, 0, 0});
    memcpy(y + base, yl, sizeof(double) * nloc);
}

static int setup(mesh_t *m, int nx, int ny, int nz, int P, const double *xv, const double *yv,
                 const double *zv, const int *bc, const double *D, const double *w)
{
    if (P < 1 || P + 1 > MAXN || nx < 1 || ny < 1 || nz < 1) return -1;
    m->n[0] = nx; m->n[1] = ny; m->n[2] = nz; m->P = P; m->np = P + 1;
    m->v[0] = xv; m->v[1] = yv; m->v[2] = zv; m->bc = bc; m->D = D; m->w = w;
    return 0;
}

/* y = A x.  nu: nodal field (ABI layout) or NULL for nu_const. */
int oracle_apply(int nx, int ny, int nz, int P, const double *xv, const double *yv, const double *zv,
                 const int *bc, const double *D, const double *w, double lambda, const double *nu,
                 double nu_const, const double *x, double *y)
{
    mesh_t m;
    if (setup(&m, nx, ny, nz, P, xv, yv, zv, bc, D, w)) return -1;
    const long ne = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (long el = 0; el < ne; ++el) {
        int e[3] = {(int)(el % nx), (int)((el / nx) % ny), (int)(el / ((long)nx * ny))};
        element_apply(&m, e, lambda, nu, nu_const, x, y);
    }
    return 0;
}

/* diag(A), read off the rows assembled by element_apply:
     lambda J W + sum_d J g_d^2 (W / w_{a_d}) sum_q w_q nu(q) D_{q a_d}^2
   plus, on a face layer with face-node weight omega and own nu:
     high face (a_d = P): omega (sigma - nu g D_PP)  interior/periodic,
                          omega (sigma - 2 nu g D_PP) Dirichlet;
     low face  (a_d = 0): omega (sigma + nu g D_00)  interior/periodic,
                          omega (sigma + 2 nu g D_00) Dirichlet.
   When a periodic axis has a single element the element is its own
   neighbour, and the far trace and far normal derivative of both of its
   faces along that axis touch the row's own node: -omega nu_n g D_0P on the
   high layer and +omega nu_n g D_P0 on the low layer, nu_n being nu at the
   opposite layer of the same line (half from each of the two faces). */
int oracle_diag(int nx, int ny, int nz, int P, const double *xv, const double *yv, const double *zv,
                const int *bc, const double *D, const double *w, double lambda, const double *nu,
                double nu_const, double *diag)
{
    mesh_t m;
    if (setup(&m, nx, ny, nz, P, xv, yv, zv, bc, D, w)) return -1;
    const long ne = (long)nx * ny * nz;
    const int np = P + 1;
#pragma omp parallel for schedule(static)
    for (long el = 0; el < ne; ++el) {
        int e[3] = {(int)(el % nx), (int)((el / nx) % ny), (int)(el / ((long)nx * ny))};
        double h[3], g[3];
        for (int d = 0; d < 3; ++d) { h[d] = extent(&m, d, e[d]); g[d] = 2.0 / h[d]; }
        const double J = h[0] * h[1] * h[2] / 8.0;
        int a[3];
        for (a[2] = 0; a[2] < np; ++a[2])
            for (a[1] = 0; a[1] < np; ++a[1])
                for (a[0] = 0; a[0] < np; ++a[0]) {
                    size_t gi = node_index(&m, e, a);
                    double W = w[a[0]] * w[a[1]] * w[a[2]];
                    double s = lambda * J * W;
                    for (int d = 0; d < 3; ++d) {
                        int b[3] = {a[0], a[1], a[2]};
                        double acc = 0.0;
                        for (int q = 0; q < np; ++q) {
                            b[d] = q;
                            acc += w[q] * nu_at(nu, nu_const, node_index(&m, e, b)) * D[q * np + a[d]] * D[q * np + a[d]];
                        }
                        s += J * g[d] * g[d] * (W / w[a[d]]) * acc;
                        if (a[d] != 0 && a[d] != P) continue;
                        const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
                        const double omega = w[a[t1]] * w[a[t2]] * h[t1] * h[t2] / 4.0;
                        const double nuo = nu_at(nu, nu_const, gi);
                        for (int side = -1; side <= 1; side += 2) {
                            if ((side > 0 && a[d] != P) || (side < 0 && a[d] != 0)) continue;
                            int nb[3];
                            int interior = neighbour(&m, e, d, side, nb);
                            const double Dff = D[a[d] * np + a[d]];
                            if (interior) {
                                int an[3] = {a[0], a[1], a[2]};
                                an[d] = (side > 0) ? 0 : P;
                                double nun = nu_at(nu, nu_const, node_index(&m, nb, an));
                                double sigma = fmax(nuo, nun) * np * np / fmin(h[d], extent(&m, d, nb[d]));
                                const double sgn = (side > 0) ? -1.0 : 1.0;
                                s += omega * (sigma + sgn * nuo * g[d] * Dff);
                                if (nb[0] == e[0] && nb[1] == e[1] && nb[2] == e[2]) {
                                    /* self-neighbour: the far trace derivative includes this node */
                                    if (side > 0) s += -omega * nun * g[d] * D[0 * np + P];
                                    else          s += omega * nun * g[d] * D[P * np + 0];
                                }
                            } else if (m.bc[d] == 1) {
                                const double sgn = (side > 0) ? -1.0 : 1.0;
                                double sigma = nuo * np * np / h[d];
                                s += omega * (sigma + 2.0 * sgn * nuo * g[d] * Dff);
                            }
                        }
                    }
                    diag[gi] = s;
                }
    }
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
