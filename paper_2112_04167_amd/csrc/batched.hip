// Batched implicit-stage solve in one persistent, cooperative launch.
//
// One IMEX Runge-Kutta stage (arXiv 2112.04167, Alg. 3) solves a pressure
// Poisson problem and three velocity Helmholtz problems on the same mesh.
// Here they are solved together, each with its own scalars, stopping test
// (Sec. 4: relative RMS residual at the collocation points) and retirement,
// in one kernel that never returns to the host.
//
// Method per system (inner precision TI: FP32 in the mixed mode, FP64
// otherwise): Jacobi-preconditioned CG on A_TI, with residual replacement
// (van der Vorst & Ye 2000; the "reliable updates" of mixed-precision CG).
// The inner vectors hold a correction x_TI and the residual scaled by a
// power of two s.  When the recurrence residual has dropped by the factor
// delta since the last replacement, or claims convergence, the correction
// is flushed into the FP64 solution, the residual is recomputed in FP64
// (r = b - A_64 x_64, the stopping test is taken on it), and the recurrence
// continues from that residual with the same search direction rescaled, so
// the Krylov space is kept instead of restarting as plain iterative
// refinement would.
//
// Grid barrier.  A cooperative-groups grid barrier on this chip costs tens
// of microseconds, growing with the work-group count: every work-group
// writes back its XCD's L2 and arrives on one device-scope counter.  Here
// the work-groups of an XCD (identified from the hardware XCC_ID register at
// start-up) first meet on a counter in their shared L2; the last arrival
// writes the XCD's L2 back once and arrives on the global counter; the last
// XCD releases a global flag, and every work-group acquires (invalidates
// its L1 and the XCD's non-coherent L2 lines) once it sees the flag.
// Reductions ride on the barrier: each work-group publishes its
// partial sums before arriving and, once released, adds all work-groups'
// partials in a fixed order, so every work-group holds bitwise identical
// scalars and takes the same branches.  Every wait has a spin
// limit that raises an error flag instead of hanging.
//
// Work decomposition: in each phase the work items are (system, element
// group) pairs of the systems taking part, dealt round-robin to the resident
// work-groups in the XCD-aware group order of the stand-alone apply.  The
// number of resident work-groups per CU is chosen by a small autotuner that
// times each candidate on the actual batch.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "apply_core.h"
#include "batched.h"
#include "dg_internal.h"
#include "kernels.h"

namespace cgrp = cooperative_groups;

namespace dg {

namespace {

constexpr int kXcdIds = 16;                // XCC_ID values tracked
constexpr unsigned kSpinLimit = 1u << 22;  // polls before a wait gives up

// ------------------------------------------------------------ grid barrier

struct SyncBlock {
    unsigned reg[kXcdIds * 64];    // work-groups per XCD (registration)
    unsigned cnt[kXcdIds * 64];    // XCD-local arrivals
    unsigned gcnt[64];             // XCDs arrived
    unsigned gflag[64];            // generation released by the last XCD
    unsigned err[64];              // a wait hit its spin limit
};

struct SyncArea {
    SyncBlock sb;
};

struct BarCtx {
    int xcc, nx;     // this work-group's XCD and the number of work-groups on it
    unsigned nxa;    // XCDs holding work-groups
    unsigned gen;    // barrier generation
    int parity;      // partial-sum buffer in use
    int err;         // a wait of this work-group gave up (spin limit or error flag)
};

__device__ __forceinline__ unsigned hw_xcc_id()
{
    unsigned v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return v & (kXcdIds - 1);
}

// acquire at device scope: drop this CU's L1 and the XCD's non-coherent L2
// lines (a work-group-scope invalidate leaves the L1 in place)
__device__ __forceinline__ void acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

__device__ __forceinline__ unsigned ld_agent(const unsigned *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ bool spin_ne(const unsigned *flag, unsigned gen, unsigned *err)
{
    for (unsigned k = 0;; ++k) {
        if (ld_agent(flag) != gen) return true;
        if ((k & 255u) == 255u && ld_agent(err)) return false;
        if (k > kSpinLimit) {
            __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Once per launch: count the work-groups on each XCD.
__device__ void grid_register(SyncArea *sa, BarCtx &bc, cgrp::grid_group &grid)
{
    if (threadIdx.x == 0) {
        const unsigned x = hw_xcc_id();
        bc.xcc = (int)x;
        __hip_atomic_fetch_add(&sa->sb.reg[x * 64], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    grid.sync();
    if (threadIdx.x == 0) {
        bc.nx = (int)ld_agent(&sa->sb.reg[bc.xcc * 64]);
        unsigned n = 0;
        for (int y = 0; y < kXcdIds; ++y) n += ld_agent(&sa->sb.reg[y * 64]) ? 1u : 0u;
        bc.nxa = n;
        bc.gen = 0;
        bc.parity = 0;
        bc.err = 0;
    }
    __syncthreads();
}

// Grid barrier with an optional sum of ncomp values per work-group.
// mine[0..ncomp): this work-group's values (LDS, final before the call);
// tot[0..ncomp): the grid totals on return (LDS).  part: [2][slots][nblk].
// After the barrier every work-group adds all work-groups' values itself, in
// work-group order, so all copies of the totals are bitwise identical.
__device__ void grid_reduce(SyncArea *sa, double *part, BarCtx &bc, const double *mine, double *tot,
                            int ncomp, double *sh)
{
    const int tid = threadIdx.x, nblk = gridDim.x;
    const int par = bc.parity;
    double *pp = part + (size_t)par * kBatchSlots * nblk;
    if (tid < ncomp) pp[(size_t)tid * nblk + blockIdx.x] = mine[tid];
    // every thread's stores have reached L2 before the work-group arrives
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    SyncBlock *sb = &sa->sb;
    if (tid == 0) {
        const int x = bc.xcc;
        const unsigned gen = bc.gen;
        const unsigned prev =
            __hip_atomic_fetch_add(&sb->cnt[x * 64], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (prev == (unsigned)bc.nx - 1) {
            // the whole XCD has arrived: publish its data device-wide once,
            // then arrive globally
            __hip_atomic_store(&sb->cnt[x * 64], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const unsigned p2 = __hip_atomic_fetch_add(&sb->gcnt[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            if (p2 == bc.nxa - 1) {
                __hip_atomic_store(&sb->gcnt[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&sb->gflag[0], gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (!spin_ne(&sb->gflag[0], gen, sb->err)) bc.err = 1;
        acquire_agent();
        bc.gen = gen + 1;
        bc.parity = par ^ 1;
    }
    __syncthreads();
    const int nw = (blockDim.x + 63) >> 6;
    for (int k0 = 0; k0 < ncomp; k0 += 16) {
        double v[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) v[c] = 0.0;
        for (int b = tid; b < nblk; b += blockDim.x)
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (k0 + c < ncomp) v[c] += pp[(size_t)(k0 + c) * nblk + b];
#pragma unroll
        for (int c = 0; c < 16; ++c)
            if (k0 + c < ncomp)
                for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_down(v[c], off, 64);
        if ((tid & 63) == 0)
#pragma unroll
            for (int c = 0; c < 16; ++c) sh[c * 16 + (tid >> 6)] = v[c];
        __syncthreads();
        if (tid < 16 && k0 + tid < ncomp) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += sh[tid * 16 + w];
            tot[k0 + tid] = s;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- the solver

template <typename TI>
struct BSys {
    double *x64, *b64, *r64;
    const double *rhs, *nu64;
    TI *x, *r, *p, *q, *u, *s;  // q holds w = A u
    const TI *d;  // 1 / diag(A_TI)
    const TI *nu;
    double lambda;
    int bc[3];
    int singular;
};

struct BResult {
    double bnorm2, res64;
    int status, iters, replaced, pad;
};

template <typename TI>
struct BArgs {
    BSys<TI> sys[kMaxBatch];
    BResult *res;
    SyncArea *sa;
    double *partial;
    Geo<double> g64;
    Geo<TI> gi;
    const int *order;
    int nel, ngroups, nsys, weak, maxit, max_replace, handoff;
    double tol, delta, mass_mean;
};

// per-system scalars; every work-group holds an identical copy
struct SysSt {
    double bnorm2, tol2, res64;
    double mean_b;              // singular: mean removed from the load
    double s, s_new, s_old;     // inner scaling (power of two): true = s * stored
    double gamma, alpha, coef;  // r.u of the step that made p, its alpha, and the
                                // coefficient of the old p and s in the next update
    double gamma_fresh;         // r.u right after a replacement
    double us, ps;              // right after a replacement: u.s, p.s (old p, s)
    double mw, sum_u;           // singular: mean of w = A u removed from s; sum u
    double res2, ref2;          // recurrence ||M^-1 r||^2 (scaled), at the last replacement
    double mean64;              // singular: mean removed from the FP64 residual
    double sum_invd, sum_invM2; // singular: sum 1/diag, sum 1/M^2
    double shift;
    int status, done, iters, replaced, repl;
    int fresh;                  // 2: just set up, 1: just replaced, 0: in the recurrence
};

// Group sizes: the inner-precision phases use the kernels' groups of EB
// elements; the FP64 residual of an FP32 solve uses groups of EBH elements so
// that its LDS fits in the FP32 buffers (it runs rarely).
template <int P, typename TI>
struct BShape {
    static constexpr int EB = Shape<P>::EB;
    static constexpr int EBH = sizeof(TI) == 8 ? EB : (EB + 1) / 2;
    static constexpr int E3 = Lds<P>::E3;
    static constexpr size_t VB = (size_t)EB * E3 * sizeof(TI) > (size_t)EBH * E3 * 8
                                     ? (size_t)EB * E3 * sizeof(TI)
                                     : (size_t)EBH * E3 * 8;
    static constexpr size_t GB = EB * sizeof(ElGeo<TI>) > EBH * sizeof(ElGeo<double>)
                                     ? EB * sizeof(ElGeo<TI>)
                                     : EBH * sizeof(ElGeo<double>);
};

template <int P, typename TI>
struct BLds {
    using BS = BShape<P, TI>;
    alignas(16) unsigned char xs[BS::VB], ys[BS::VB], nus[BS::VB];
    alignas(16) unsigned char geo[BS::GB];
    double sh[16 * 16];
    double acc[kBatchSlots];
    double tot[kBatchSlots];
};


__device__ __forceinline__ double pow2_near(double v)
{
    if (!(v > 0.0) || !isfinite(v)) return 1.0;
    return exp2(rint(log2(v)));
}

// per-thread node loop of one element group: f(global index, GLL mass, 1/mass)
template <int P, typename F>
__device__ __forceinline__ void group_nodes(int grp, int nel, const Geo<double> &g, F &&f)
{
    using S = Shape<P>;
    const int tid = threadIdx.x;
    const int el_loc = tid / S::NL;
    const int l = tid - el_loc * S::NL;
    const int el = grp * S::EB + el_loc;
    if (tid >= S::NT || el >= nel) return;
    const int ex = el % g.n[0], r = el / g.n[0], ey = r % g.n[1], ez = r / g.n[1];
    const double Jw = g.h[0][ex] * g.h[1][ey] * g.h[2][ez] * 0.125 * kGll<P>.w[l % S::n] *
                      kGll<P>.w[l / S::n];
    const double iJw = 1.0 / Jw;
#pragma unroll
    for (int c = 0; c < S::n; ++c)
        f((size_t)el * S::N3 + (size_t)c * S::NL + l, Jw * kGll<P>.w[c], iJw * (1.0 / kGll<P>.w[c]));
}

// the same per line: f(index of node (a,b,0) of the thread's line, 1/(J w_a w_b));
// the caller walks c = 0..P (stride (P+1)^2), loading all values of the line
// before storing any, so that the loads are in flight together
template <int P, typename F>
__device__ __forceinline__ void group_lines(int grp, int nel, const Geo<double> &g, F &&f)
{
    using S = Shape<P>;
    const int tid = threadIdx.x;
    const int el_loc = tid / S::NL;
    const int l = tid - el_loc * S::NL;
    const int el = grp * S::EB + el_loc;
    if (tid >= S::NT || el >= nel) return;
    const int ex = el % g.n[0], r = el / g.n[0], ey = r % g.n[1], ez = r / g.n[1];
    const double Jw = g.h[0][ex] * g.h[1][ey] * g.h[2][ez] * 0.125 * kGll<P>.w[l % S::n] *
                      kGll<P>.w[l / S::n];
    f((size_t)el * S::N3 + l, 1.0 / Jw);
}

template <typename T>
__device__ __forceinline__ ApplyArgs<T> sys_apply_args(const Geo<T> &g, const int *bc, int nel, int G,
                                                       const int *order, const T *x, T *y,
                                                       const T *nu, double lambda, const T *b)
{
    ApplyArgs<T> a{};
    a.x = x;
    a.y = y;
    a.nu = nu;
    a.nu_c = (T)1;
    a.lambda = (T)lambda;
    a.geo = g;
    for (int d = 0; d < 3; ++d) a.geo.bc[d] = bc[d];
    a.nel = nel;
    a.ngroups = G;
    a.order = order;
    a.b = b;
    return a;
}

template <int P, typename TI>
__device__ __forceinline__ void batched_body(BArgs<TI> &B)
{
    using S = Shape<P>;
    using BS = BShape<P, TI>;
    __shared__ BLds<P, TI> L;
    __shared__ SysSt st[kMaxBatch];
    __shared__ BarCtx bc;
    __shared__ int list[kMaxBatch];
    __shared__ int nlist;
    __shared__ int sh_flag;
    cgrp::grid_group grid = cgrp::this_grid();
    const int tid = threadIdx.x;
    const int G = B.ngroups, nel = B.nel, ns = B.nsys;
    const double N = (double)nel * S::N3;

    for (int k = tid; k < (int)(kMaxBatch * sizeof(SysSt) / sizeof(int)); k += blockDim.x)
        reinterpret_cast<int *>(st)[k] = 0;
    grid_register(B.sa, bc, grid);

    // systems for which pred(s) holds, in index order (identical in every
    // work-group); returns their number
    auto make_list = [&](auto pred) -> int {
        if (tid == 0) {
            int k = 0;
            for (int s = 0; s < ns; ++s)
                if (pred(st[s])) list[k++] = s;
            nlist = k;
        }
        __syncthreads();
        return nlist;
    };
    auto clear_acc = [&]() {
        if (tid < kBatchSlots) L.acc[tid] = 0.0;
        __syncthreads();
    };
    // work items (slot in the list, system, element group)
    auto items = [&](int n, auto &&f) {
        for (int w = blockIdx.x; w < n * G; w += gridDim.x) {
            const int slot = w / G;
            const int s = __builtin_amdgcn_readfirstlane(list[slot]);
            const int g = xcd_remap(w % G, G);
            f(slot, s, B.order ? B.order[g] : g);
        }
    };
    auto add_acc = [&](auto &v, int slot) {
        constexpr int K = sizeof(v) / sizeof(double);
        block_sum<K>(v, L.sh);
        if (tid == 0)
#pragma unroll
            for (int c = 0; c < K; ++c) L.acc[slot * K + c] += v[c];
    };
    // sum the accumulators of n systems (k components each, the k of the
    // phase's add_acc) over the grid,
    // then fin(system, totals) on thread 0 in list order
    auto reduce = [&](int n, int k, auto &&fin) {
        grid_reduce(B.sa, B.partial, bc, L.acc, L.tot, n * k, L.sh);
        if (tid == 0)
            for (int slot = 0; slot < n; ++slot) fin(st[list[slot]], list[slot], &L.tot[slot * k]);
        __syncthreads();
    };
    auto barrier = [&]() { grid_reduce(B.sa, B.partial, bc, L.acc, L.tot, 0, L.sh); };

    TI *xs = reinterpret_cast<TI *>(L.xs), *ys = reinterpret_cast<TI *>(L.ys),
       *nus = reinterpret_cast<TI *>(L.nus);
    ElGeo<TI> *geo = reinterpret_cast<ElGeo<TI> *>(L.geo);

    // ---- set-up 1: b = M f (or f), x = 0; sum b, sum b^2
    int n = make_list([](const SysSt &) { return true; });
    clear_acc();
    items(n, [&](int slot, int s, int g) {
        const BSys<TI> &Y = B.sys[s];
        double v[2] = {0.0, 0.0};
        group_nodes<P>(g, nel, B.g64, [&](size_t gi, double m, double) {
            const double bb = B.weak ? Y.rhs[gi] : m * Y.rhs[gi];
            Y.b64[gi] = bb;
            Y.x64[gi] = 0.0;
            v[0] += bb;
            v[1] += bb * bb;
        });
        add_acc(v, slot);
    });
    reduce(n, 2, [&](SysSt &y, int s, const double *t) {
        y.status = DG_OK;
        y.mean_b = B.sys[s].singular ? t[0] / N : 0.0;
        const double ms = t[1] / N - y.mean_b * y.mean_b;
        y.s = pow2_near(sqrt(ms > 0.0 ? ms : t[1] / N));
        if (!isfinite(t[1])) {
            y.status = DG_ERR_NONFINITE;
            y.done = 1;
        }
    });

    // ---- set-up 2: project b (singular); inner r = b / s, u = r/diag, x = p = s = 0
    n = make_list([](const SysSt &y) { return !y.done; });
    clear_acc();
    items(n, [&](int slot, int s, int g) {
        const BSys<TI> &Y = B.sys[s];
        const double mb = st[s].mean_b, is = 1.0 / st[s].s;
        double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        group_nodes<P>(g, nel, B.g64, [&](size_t gi, double, double im) {
            double bb = Y.b64[gi];
            if (Y.singular) {
                bb -= mb;
                Y.b64[gi] = bb;
            }
            const TI r = (TI)(bb * is);
            const TI u = r * Y.d[gi];
            Y.r[gi] = r;
            Y.u[gi] = u;
            Y.x[gi] = (TI)0;
            Y.p[gi] = (TI)0;
            Y.s[gi] = (TI)0;
            const double rm = bb * im, rs = (double)r * im;
            v[0] += rm * rm;
            v[1] += im * im;
            v[2] += (double)Y.d[gi];
            v[3] += (double)r * (double)u;
            v[4] += rs * rs;
            v[5] += (double)u;
        });
        add_acc(v, slot);
    });
    reduce(n, 6, [&](SysSt &y, int, const double *t) {
        y.bnorm2 = t[0];
        y.res64 = t[0];
        y.tol2 = B.tol * B.tol * t[0];
        y.sum_invM2 = t[1];
        y.sum_invd = t[2];
        y.gamma = t[3];
        y.res2 = y.ref2 = t[4];
        y.sum_u = t[5];
        y.fresh = 2;  // no previous direction
        if (!isfinite(t[0]) || !isfinite(t[3])) {
            y.status = DG_ERR_NONFINITE;
            y.done = 1;
        } else if (!(t[0] > 0.0)) {
            y.done = 1;  // b = 0: x = 0
        }
    });

    // Jacobi-PCG with one reduction per iteration (the Chronopoulos-Gear
    // arrangement): one element-wise phase (new direction p = u + beta p,
    // s = A p by the same recurrence, x, r, and u = r/diag), then w = A u.
    // The dot products of both phases are reduced together: gamma = r.u,
    // ||M^-1 r||^2, and the pieces of (p', A p') = (p', s') for the next
    // direction p' = u + beta' p, s' = w + beta' s, taken from the actual
    // vectors (u.w, u.s, p.s; p.w = u.s by symmetry) rather than from the
    // orthogonality relations of the textbook recurrence, which decay in
    // FP32.  An iteration costs one grid-wide reduction and one plain barrier.
    for (;;) {
        // bc.err: a barrier wait of this work-group gave up; the others find
        // the device flag in their own waits
        n = make_list([](const SysSt &y) { return !y.done; });
        if (n == 0 || bc.err) break;
        if (B.handoff && n == 1 && B.nsys > 1) {
            // a single system left: its iterations are cheaper as ordinary
            // kernels than behind two grid barriers each, so the launch ends
            // here.  Flush its correction into x_64 (the current solution, from
            // which the caller continues) and report it as handed off.
            items(1, [&](int, int s, int g) {
                const BSys<TI> &Y = B.sys[s];
                const double sc = st[s].s;
                group_lines<P>(g, nel, B.g64, [&](size_t base, double) {
                    constexpr int n = S::n, NL = S::NL;
                    double xd[n];
                    TI xv[n];
#pragma unroll
                    for (int c = 0; c < n; ++c) {
                        xd[c] = Y.x64[base + (size_t)c * NL];
                        xv[c] = Y.x[base + (size_t)c * NL];
                    }
#pragma unroll
                    for (int c = 0; c < n; ++c) Y.x64[base + (size_t)c * NL] = fma(sc, (double)xv[c], xd[c]);
                });
            });
            barrier();
            if (tid == 0) {
                st[list[0]].status = kBatchHandoff;
                st[list[0]].done = 1;
            }
            __syncthreads();
            break;
        }
        clear_acc();

        // ---- p = u + beta p, s = (w - mean w) + beta s, x += alpha p,
        //      r -= alpha s, u = r/diag; gamma, ||M^-1 r||^2, sum u
        //      (systems just set up or replaced start at w = A u)
        bool any_e = false;
        if (tid == 0) {
            int k = 0;
            for (int i = 0; i < n; ++i) k += st[list[i]].fresh ? 0 : 1;
            sh_flag = k;
        }
        __syncthreads();
        any_e = sh_flag > 0;
        if (any_e) {
            items(n, [&](int slot, int s, int g) {
                if (st[s].fresh) return;
                const BSys<TI> &Y = B.sys[s];
                const TI alpha = (TI)st[s].alpha, beta = (TI)st[s].coef, mw = (TI)st[s].mw;
                double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                group_lines<P>(g, nel, B.g64, [&](size_t base, double iJw) {
                    constexpr int n = S::n, NL = S::NL;
                    TI uv[n], pv[n], wv[n], sv[n], xv[n], rv[n], dv[n];
#pragma unroll
                    for (int c = 0; c < n; ++c) {
                        const size_t gi = base + (size_t)c * NL;
                        uv[c] = Y.u[gi];
                        pv[c] = Y.p[gi];
                        wv[c] = Y.q[gi];
                        sv[c] = Y.s[gi];
                        xv[c] = Y.x[gi];
                        rv[c] = Y.r[gi];
                        dv[c] = Y.d[gi];
                    }
#pragma unroll
                    for (int c = 0; c < n; ++c) {
                        const size_t gi = base + (size_t)c * NL;
                        const TI p = fma(beta, pv[c], uv[c]);
                        const TI sd = fma(beta, sv[c], wv[c] - mw);
                        const TI r = fma(-alpha, sd, rv[c]);
                        const TI u = r * dv[c];
                        Y.p[gi] = p;
                        Y.s[gi] = sd;
                        Y.x[gi] = fma(alpha, p, xv[c]);
                        Y.r[gi] = r;
                        Y.u[gi] = u;
                        const double rm = (double)r * (iJw * (1.0 / kGll<P>.w[c]));
                        v[0] += (double)r * (double)u;
                        v[1] += rm * rm;
                        v[2] += (double)u;
                        v[3] += (double)u * (double)sd;
                        v[4] += (double)p * (double)sd;
                    }
                });
                add_acc(v, slot);
            });
            barrier();
        }

        // ---- w = A u; w.u, sum w
        items(n, [&](int slot, int s, int g) {
            const BSys<TI> &Y = B.sys[s];
            ApplyArgs<TI> a = sys_apply_args<TI>(B.gi, Y.bc, nel, G, B.order, Y.u, Y.q, Y.nu, Y.lambda, nullptr);
            double red[4];
            constexpr bool LZ = apply_lazy<P, TI>();
            if (Y.nu)
                apply_group<P, TI, true, EPI_CG, S::EB, LZ, true>(a, g, xs, ys, nus, geo, red);
            else
                apply_group<P, TI, false, EPI_CG, S::EB, LZ, true>(a, g, xs, ys, nus, geo, red);
            double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, red[0], red[1]};
            add_acc(v, slot);
        });
        reduce(n, 7, [&](SysSt &y, int s, const double *t) {
            // t: [0] r.u [1] ||M^-1 r||^2 [2] sum u [3] u.s [4] p.s (this
            //    step's element-wise phase; after a set-up or a replacement
            //    they come from that phase) [5] u.w [6] sum w
            double g1, r2, su, us, ps;
            if (y.fresh) {
                g1 = y.fresh == 1 ? y.gamma_fresh : y.gamma;
                r2 = y.res2;
                su = y.sum_u;
                us = y.us;
                ps = y.ps;
            } else {
                g1 = t[0];
                r2 = t[1] < 0.0 ? 0.0 : t[1];
                su = t[2];
                us = t[3];
                ps = t[4];
                y.iters += 1;
            }
            const double mw = B.sys[s].singular ? t[6] / N : 0.0;
            // with w - mean w; p.(A u) = u.(A p) = u.s (s: the recurrence for A p)
            const double uw = t[5] - mw * su, pw = us;
            if (!isfinite(g1) || !isfinite(r2) || !isfinite(uw)) {
                y.status = DG_ERR_NONFINITE;
                y.done = 1;
                return;
            }
            if (!y.fresh) {
                y.res2 = r2;
                if (r2 * y.s * y.s <= y.tol2 || r2 <= B.delta * B.delta * y.ref2 || y.iters >= B.maxit) {
                    y.repl = 1;  // keep gamma of the step that made p
                    return;
                }
            }
            // coefficient of the old p and s (still in the scaling of the
            // previous replacement) in p' = u + c p, s' = (w - mean w) + c s
            double coef = 0.0;
            if (y.fresh == 1)
                coef = (g1 / y.gamma) * (y.s / y.s_old);
            else if (!y.fresh)
                coef = g1 / y.gamma;
            // (p', A p') = (p', s') from this step's vectors
            const double den = uw + coef * (us + pw) + coef * coef * ps;
            if (!(den > 0.0)) {
                y.status = DG_ERR_NOT_SPD;
                y.done = 1;
                return;
            }
            y.alpha = g1 / den;
            y.coef = coef;
            y.gamma = g1;
            y.mw = mw;
            y.sum_u = su;
            y.fresh = 0;
        });

        n = make_list([](const SysSt &y) { return !y.done && y.repl; });
        if (n > 0) {
            // ---- flush: x_64 += s x_TI, x_TI = 0
            items(n, [&](int, int s, int g) {
                const BSys<TI> &Y = B.sys[s];
                const double sc = st[s].s;
                group_lines<P>(g, nel, B.g64, [&](size_t base, double) {
                    constexpr int n = S::n, NL = S::NL;
                    double xd[n];
                    TI xv[n];
#pragma unroll
                    for (int c = 0; c < n; ++c) {
                        xd[c] = Y.x64[base + (size_t)c * NL];
                        xv[c] = Y.x[base + (size_t)c * NL];
                    }
#pragma unroll
                    for (int c = 0; c < n; ++c) {
                        Y.x64[base + (size_t)c * NL] = fma(sc, (double)xv[c], xd[c]);
                        Y.x[base + (size_t)c * NL] = (TI)0;
                    }
                });
            });
            barrier();
            // ---- FP64 residual r_64 = b - A_64 x_64 and the stopping test
            clear_acc();
            {
                constexpr int EBH = BS::EBH;
                const int GH = (nel + EBH - 1) / EBH;
                double *xd = reinterpret_cast<double *>(L.xs), *yd = reinterpret_cast<double *>(L.ys),
                       *nd = reinterpret_cast<double *>(L.nus);
                ElGeo<double> *gd = reinterpret_cast<ElGeo<double> *>(L.geo);
                for (int w = blockIdx.x; w < n * GH; w += gridDim.x) {
                    const int slot = w / GH;
                    const int s = __builtin_amdgcn_readfirstlane(list[slot]);
                    int g = xcd_remap(w % GH, GH);
                    if (EBH == S::EB && B.order) g = B.order[g];
                    const BSys<TI> &Y = B.sys[s];
                    ApplyArgs<double> a = sys_apply_args<double>(B.g64, Y.bc, nel, GH, nullptr, Y.x64,
                                                                 Y.r64, Y.nu64, Y.lambda, Y.b64);
                    double red[4];
                    if (Y.nu64)
                        apply_group<P, double, true, EPI_RESID, EBH, true, true>(a, g, xd, yd, nd, gd, red);
                    else
                        apply_group<P, double, false, EPI_RESID, EBH, true, true>(a, g, xd, yd, nd, gd, red);
                    add_acc(red, slot);
                }
            }
            reduce(n, 4, [&](SysSt &y, int s, const double *t) {
                double res = t[0], m = 0.0;
                if (B.sys[s].singular) {
                    m = t[1] / N;
                    res = t[0] - 2.0 * m * t[2] + m * m * t[3];
                }
                if (res < 0.0) res = 0.0;
                y.res64 = res;
                y.mean64 = m;
                y.replaced += 1;
                if (!isfinite(res)) {
                    y.status = DG_ERR_NONFINITE;
                    y.done = 1;
                } else if (res <= y.tol2) {
                    y.done = 1;
                } else if (y.iters >= B.maxit || y.replaced >= B.max_replace) {
                    y.status = DG_NOT_CONVERGED;
                    y.done = 1;
                } else {
                    y.s_new = pow2_near(sqrt(res / N) * B.mass_mean);
                }
                if (y.done) y.repl = 0;
            });
            n = make_list([](const SysSt &y) { return !y.done && y.repl; });
            if (n > 0) {
                // ---- replace: r_TI = (r_64 - mean) / s_new, u = r/diag
                clear_acc();
                items(n, [&](int slot, int s, int g) {
                    const BSys<TI> &Y = B.sys[s];
                    const double m = st[s].mean64, is = 1.0 / st[s].s_new;
                    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
                    group_lines<P>(g, nel, B.g64, [&](size_t base, double iJw) {
                        constexpr int n = S::n, NL = S::NL;
                        double rr[n];
                        TI dv[n], pv[n], sv[n];
#pragma unroll
                        for (int c = 0; c < n; ++c) {
                            rr[c] = Y.r64[base + (size_t)c * NL];
                            dv[c] = Y.d[base + (size_t)c * NL];
                            pv[c] = Y.p[base + (size_t)c * NL];
                            sv[c] = Y.s[base + (size_t)c * NL];
                        }
#pragma unroll
                        for (int c = 0; c < n; ++c) {
                            const TI r = (TI)((rr[c] - m) * is);
                            const TI u = r * dv[c];
                            Y.r[base + (size_t)c * NL] = r;
                            Y.u[base + (size_t)c * NL] = u;
                            const double rm = (double)r * (iJw * (1.0 / kGll<P>.w[c]));
                            v[0] += (double)r * (double)u;
                            v[1] += rm * rm;
                            v[2] += (double)u;
                            v[3] += (double)u * (double)sv[c];
                            v[4] += (double)pv[c] * (double)sv[c];
                        }
                    });
                    add_acc(v, slot);
                });
                reduce(n, 5, [&](SysSt &y, int, const double *t) {
                    y.gamma_fresh = t[0];
                    y.res2 = y.ref2 = t[1];
                    y.sum_u = t[2];
                    y.us = t[3];
                    y.ps = t[4];
                    y.s_old = y.s;
                    y.s = y.s_new;
                    y.repl = 0;
                    y.fresh = 1;
                });
            }
        }
    }

    // ---- singular systems: remove the M-weighted mean of x
    n = make_list([&](const SysSt &y) { return y.status >= 0 && y.bnorm2 > 0.0; });
    {
        // keep only singular systems (list order preserved)
        if (tid == 0) {
            int k = 0;
            for (int i = 0; i < nlist; ++i)
                if (B.sys[list[i]].singular) list[k++] = list[i];
            nlist = k;
        }
        __syncthreads();
        n = nlist;
    }
    if (n > 0 && !bc.err) {
        clear_acc();
        items(n, [&](int slot, int s, int g) {
            const BSys<TI> &Y = B.sys[s];
            double v[2] = {0.0, 0.0};
            group_nodes<P>(g, nel, B.g64, [&](size_t gi, double m, double) {
                v[0] += m * Y.x64[gi];
                v[1] += m;
            });
            add_acc(v, slot);
        });
        reduce(n, 2, [&](SysSt &y, int, const double *t) { y.shift = t[1] > 0.0 ? t[0] / t[1] : 0.0; });
        items(n, [&](int, int s, int g) {
            const BSys<TI> &Y = B.sys[s];
            const double sh = st[s].shift;
            group_nodes<P>(g, nel, B.g64, [&](size_t gi, double, double) { Y.x64[gi] -= sh; });
        });
    }
    if (blockIdx.x == 0 && tid == 0)
        for (int s = 0; s < ns; ++s) {
            BResult r;
            r.bnorm2 = st[s].bnorm2;
            r.res64 = st[s].res64;
            r.status = st[s].status;
            r.iters = st[s].iters;
            r.replaced = st[s].replaced;
            r.pad = 0;
            B.res[s] = r;
        }
}

// The FP32 instantiation asks for the occupancy of the stand-alone FP32
// apply (4 waves/SIMD), so that its frequent FP32 phases keep it; its rare
// FP64 residual phase loads neighbour lines lazily to fit that budget.
template <int P>
__global__ void __launch_bounds__(Shape<P>::NTP, 4) k_batched_f32(BArgs<float> B)
{
    batched_body<P, float>(B);
}

template <int P>
__global__ void __launch_bounds__(Shape<P>::NTP) k_batched_f64(BArgs<double> B)
{
    batched_body<P, double>(B);
}

template <int P, typename TI>
const void *kernel_ptr()
{
    if constexpr (sizeof(TI) == 4)
        return reinterpret_cast<const void *>(&k_batched_f32<P>);
    else
        return reinterpret_cast<const void *>(&k_batched_f64<P>);
}

template <typename TI>
const void *kernel_for(int P)
{
    switch (P) {
        case 3: return kernel_ptr<3, TI>();
        case 4: return kernel_ptr<4, TI>();
        case 5: return kernel_ptr<5, TI>();
        case 6: return kernel_ptr<6, TI>();
        case 7: return kernel_ptr<7, TI>();
        case 8: return kernel_ptr<8, TI>();
    }
    return nullptr;
}

template <typename TI>
void fill_args(BArgs<TI> &B, const MeshDev &m, const BatchRequest &req)
{
    B.nsys = req.nsys;
    B.handoff = req.handoff;
    B.res = (BResult *)req.results;
    B.sa = (SyncArea *)req.sync;
    B.partial = req.partial;
    const TI *h = sizeof(TI) == 8 ? (const TI *)m.h64 : (const TI *)m.h32;
    const TI *ih = sizeof(TI) == 8 ? (const TI *)m.ih64 : (const TI *)m.ih32;
    int off = 0;
    for (int d = 0; d < 3; ++d) {
        B.g64.n[d] = B.gi.n[d] = m.n[d];
        B.g64.bc[d] = B.gi.bc[d] = m.bc[d];
        B.g64.h[d] = m.h64 + off;
        B.g64.ih[d] = m.ih64 + off;
        B.gi.h[d] = h + off;
        B.gi.ih[d] = ih + off;
        off += m.n[d];
    }
    B.order = m.order;
    B.nel = (int)m.nel;
    B.ngroups = apply_groups(m.P, m.nel);
    B.weak = req.weak;
    B.maxit = req.maxit;
    B.max_replace = req.max_replace;
    B.tol = req.tol;
    B.delta = req.delta;
    B.mass_mean = req.mass_mean;
    for (int s = 0; s < req.nsys; ++s) {
        const BatchSysDesc &D = req.sys[s];
        BSys<TI> &Y = B.sys[s];
        Y.x64 = D.x64;
        Y.b64 = D.b64;
        Y.r64 = D.r64;
        Y.rhs = D.rhs;
        Y.nu64 = D.nu64;
        Y.x = (TI *)D.xi;
        Y.r = (TI *)D.ri;
        Y.p = (TI *)D.pi;
        Y.q = (TI *)D.qi;
        Y.u = (TI *)D.ui;
        Y.s = (TI *)D.si;
        Y.d = (const TI *)D.di;
        Y.nu = (const TI *)D.nui;
        Y.lambda = D.lambda;
        for (int d = 0; d < 3; ++d) Y.bc[d] = D.bc[d];
        Y.singular = D.singular;
    }
}

// autotuned launch shape per (device, P, inner precision, nsys, mesh size)
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, long long>, int> g_tune;

}  // namespace

size_t batched_sync_bytes() { return sizeof(SyncArea); }
size_t batched_result_bytes() { return sizeof(BResult) * kMaxBatch; }
size_t batched_partial_doubles() { return (size_t)2 * kBatchSlots * kBatchMaxBlocks; }
size_t batched_sync_err_offset() { return offsetof(SyncArea, sb) + offsetof(SyncBlock, err); }

int batched_check_sync(const void *host_sync_err)
{
    if (*(const unsigned *)host_sync_err) {
        set_error("batched solve: a grid barrier wait exceeded its spin limit");
        return DG_ERR_DEVICE;
    }
    return DG_OK;
}

int batched_read_results(const void *host_results, int s, BatchSysResult *out)
{
    const BResult *r = (const BResult *)host_results + s;
    out->status = r->status;
    out->iters = r->iters;
    out->replaced = r->replaced;
    out->bnorm2 = r->bnorm2;
    out->res64 = r->res64;
    return DG_OK;
}

int batched_launch(const MeshDev &m, const BatchRequest &req, hipStream_t stream, int *blocks_per_cu)
{
    const bool f32 = req.inner_fp32;
    const void *fn = f32 ? kernel_for<float>(m.P) : kernel_for<double>(m.P);
    if (!fn) {
        set_error("polynomial degree outside 3..8");
        return DG_ERR_ARG;
    }
    int dev = 0;
    DG_HIP_CHECK(hipGetDevice(&dev));
    int coop = 0, ncu = 0;
    DG_HIP_CHECK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    DG_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (!coop) {
        set_error("device does not support cooperative launches");
        return DG_ERR_DEVICE;
    }
    const int threads = apply_threads(m.P);
    int per_cu = 0;
    DG_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0));
    if (per_cu < 1) {
        set_error("batched kernel does not fit on a compute unit");
        return DG_ERR_DEVICE;
    }
    per_cu = std::min(per_cu, kBatchMaxBlocks / ncu);

    auto run = [&](int bpc, int maxit) -> int {
        DG_HIP_CHECK(hipMemsetAsync(req.sync, 0, sizeof(SyncBlock), stream));
        const dim3 grid(ncu * bpc), block(threads);
        if (f32) {
            BArgs<float> B{};
            fill_args(B, m, req);
            B.maxit = maxit;
            void *args[] = {&B};
            DG_HIP_CHECK(hipLaunchCooperativeKernel(fn, grid, block, args, 0, stream));
        } else {
            BArgs<double> B{};
            fill_args(B, m, req);
            B.maxit = maxit;
            void *args[] = {&B};
            DG_HIP_CHECK(hipLaunchCooperativeKernel(fn, grid, block, args, 0, stream));
        }
        return DG_OK;
    };

    // autotune: time a short, fixed amount of work for every launch shape
    int bpc = 1;
    const auto key = std::make_tuple(dev, m.P, f32 ? 1 : 0, req.nsys, (long long)m.nel);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            bpc = std::min(it->second, per_cu);
        } else {
            double best = 1e300;
            hipEvent_t e0, e1;
            DG_HIP_CHECK(hipEventCreate(&e0));
            DG_HIP_CHECK(hipEventCreate(&e1));
            for (int c = 1; c <= per_cu; ++c) {
                DG_HIP_CHECK(hipEventRecord(e0, stream));
                int rc = run(c, 8);
                DG_HIP_CHECK(hipEventRecord(e1, stream));
                DG_HIP_CHECK(hipEventSynchronize(e1));
                float ms = 0.f;
                DG_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
                if (rc) return rc;
                if (ms < best) {
                    best = ms;
                    bpc = c;
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            g_tune[key] = bpc;
        }
    }
    if (blocks_per_cu) *blocks_per_cu = bpc;
    return run(bpc, req.maxit);
}

}  // namespace dg
