// Fast-diagonalisation preconditioner on the GPU: the three 1D transforms of
// z = (S (x) S (x) S) (lambda + nu Lam)^-1 (S (x) S (x) S)^T r as FP64 MFMA
// contractions along the mesh axes (gfx950, v_mfma_f64_16x16x4f64), or as
// FP32 MFMA contractions (v_mfma_f32_16x16x4f32, twice the FP64 matrix rate)
// with FP32 intermediates for the FP32 preconditioner.
//
// A mesh line along axis d has L = n_d (P+1) nodes, global 1D index
// g = e (P+1) + a.  Every line along d is multiplied by the same dense L x L
// matrix, so one transform is a product OUT = G^T IN with IN of L rows and one
// column per mesh line.  A work-group takes one bundle -- the n_d elements of
// an element column along d, whose (P+1)^2 lines it holds completely -- or a
// chunk of its columns: it stages the bundle (all L rows, NTC*16 columns) in
// LDS with coalesced loads (an element is n^3 consecutive values in the
// element-major layout), forms the products with MFMA tiles of 16 output rows
// x 16 columns (the A operand, G, streams from L2: the matrices are shared by
// all work-groups), writes the tiles back to LDS and stores the bundle with
// coalesced stores.  The z transform runs forward, divides by the eigenvalue
// sums and runs backward in one launch, since its bundle holds every z index
// of its columns.
//
// Arithmetic per node and transform: 2 L flops, against 16 bytes of HBM
// traffic (read + write), so the kernels are bound by the FP64 matrix rate
// (78.6 TFLOP/s), not by HBM, for L > ~40.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <array>
#include <type_traits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <string>

#include <sys/stat.h>

#include "fdm.h"
#include "kernels.h"

namespace dg {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// accumulator tile of one MFMA: 4 values per lane
template <typename TC>
using acc4 = typename std::conditional<std::is_same<TC, double>::value, d4, f4>::type;

// Element types of a transform launch: TI of the input vector, TO of the
// output vector, TC of the bundle in LDS, the matrices and the MFMA
// arithmetic (FP64, or FP32 for the FP32 preconditioner).
struct FdmArgs {
    const void *in;     // TI
    void *out;          // TO
    const void *G;      // TC [k][i'] Lp x Lp (the z launch: forward)
    const void *G2;     // TC, z launch: backward matrix
    const double *lam[3];
    double lambda, nu;
    const CgScalars *sc;  // done flag and mean_r (may be null)
    int sub_mean;         // subtract sc->mean_r from the input (singular residual)
    int singular;         // drop the (0,0,0) mode
    int n, nd, L, Lp;
    int nx, ny, nz;
    int F, NBc, nchunk;   // columns per bundle, per chunk, chunks per bundle
    int rs;               // LDS row stride (doubles)
};

// element-local offset o (memory order) -> (g_local = a along the axis, column f)
template <int AXIS>
__device__ __forceinline__ void split_o(int o, int n, int &ga, int &f)
{
    if (AXIS == 0) {  // o = f n + a, f = c n + b
        ga = o % n;
        f = o / n;
    } else if (AXIS == 1) {  // o = c n^2 + b n + a: g part b, f = c n + a
        const int a = o % n, q = o / n;
        ga = q % n;
        f = (q / n) * n + a;
    } else {  // o = c n^2 + f: g part c, f = b n + a
        ga = o / (n * n);
        f = o - ga * n * n;
    }
}

// bundle -> (first node of element 0 of the bundle, element stride along the axis)
template <int AXIS>
__device__ __forceinline__ void bundle_base(const FdmArgs &A, int bundle, size_t &base, size_t &se,
                                            int &i0, int &i1)
{
    const size_t n3 = (size_t)A.n * A.n * A.n;
    if (AXIS == 0) {  // bundle = ez ny + ey
        base = (size_t)bundle * A.nx * n3;
        se = n3;
        i0 = bundle % A.ny;  // ey
        i1 = bundle / A.ny;  // ez
    } else if (AXIS == 1) {  // bundle = ez nx + ex
        const int ex = bundle % A.nx, ez = bundle / A.nx;
        base = ((size_t)ez * A.ny * A.nx + ex) * n3;
        se = (size_t)A.nx * n3;
        i0 = ex;
        i1 = ez;
    } else {  // bundle = ey nx + ex
        base = (size_t)bundle * n3;
        se = (size_t)A.nx * A.ny * n3;
        i0 = bundle % A.nx;  // ex
        i1 = bundle / A.nx;  // ey
    }
}

// OUT tiles (MT row tiles per wave, NTC column tiles) = G^T B, B = the LDS
// bundle.  Wave w owns the row tiles w, w + 4, ..., w + 4 (MT - 1); a tile
// past the last row (when Lp / 16 is not a multiple of 4) reads a valid row
// of G and its result is discarded, so the loop has no branches and the
// compiler can keep the next group's fragment loads in flight while the
// current group's MFMAs run (a branch per tile made it wait for every load).
// The K loop runs in groups of 16 (4 MFMA steps of K = 4), A (from L2) and
// B (from LDS) fragments double-buffered by group.
template <int NTC, int MT, typename TC>
__device__ __forceinline__ void gemm_bundle(const TC *__restrict__ G, const TC *Bs, int rs, int Lp,
                                            acc4<TC> (&acc)[MT][NTC])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NTC; ++nt) acc[mt][nt] = acc4<TC>{0, 0, 0, 0};
    int col[MT];  // A operand column of this lane per row tile: G[k][16 T + li]
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int T = w + 4 * mt;
        col[mt] = (16 * T < Lp ? 16 * T : 0) + li;
    }
    constexpr int U = 4;
    const int ngrp = Lp / 16;
    TC a0[U][MT], a1[U][MT], b0[U][NTC], b1[U][NTC];
    auto load = [&](int g, TC (&a)[U][MT], TC (&b)[U][NTC]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = 16 * g + 4 * u + lk;
            const TC *gr = G + (size_t)k * Lp;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) a[u][mt] = gr[col[mt]];
#pragma unroll
            for (int nt = 0; nt < NTC; ++nt) b[u][nt] = Bs[k * rs + 16 * nt + li];
        }
    };
    auto mma = [&](const TC (&a)[U][MT], const TC (&b)[U][NTC]) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NTC; ++nt) {
                    if constexpr (std::is_same<TC, double>::value)
                        acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][mt], b[u][nt], acc[mt][nt], 0, 0, 0);
                    else
                        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][mt], b[u][nt], acc[mt][nt], 0, 0, 0);
                }
    };
    load(0, a0, b0);
    int g = 0;
    for (; g + 3 <= ngrp; g += 2) {  // groups g, g + 1; g + 2 exists
        load(g + 1, a1, b1);
        mma(a0, b0);
        load(g + 2, a0, b0);
        mma(a1, b1);
    }
    if (g + 2 == ngrp) {
        load(g + 1, a1, b1);
        mma(a0, b0);
        mma(a1, b1);
    } else {
        mma(a0, b0);
    }
}

// accumulator element r of a lane -> (row, column) within the 16 x 16 tile,
// checked with in-bounds probes (A operand A[lane % 16][lane / 16], B operand
// B[lane / 16][lane % 16] in both): v_mfma_f64_16x16x4f64 holds rows
// lane / 16 + 4 r, v_mfma_f32_16x16x4f32 rows 4 (lane / 16) + r
template <typename TC>
__device__ __forceinline__ int acc_row(int lane, int r)
{
    return std::is_same<TC, double>::value ? 4 * r + (lane >> 4) : 4 * (lane >> 4) + r;
}
__device__ __forceinline__ int acc_col(int lane) { return lane & 15; }

template <int NTC, int MT, typename TC>
__device__ __forceinline__ void acc_to_lds(const acc4<TC> (&acc)[MT][NTC], TC *Bs, int rs, int Lp)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
        if (16 * (w + 4 * mt) < Lp) {
            const int row0 = 16 * (w + 4 * mt);
#pragma unroll
            for (int nt = 0; nt < NTC; ++nt)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    Bs[(row0 + acc_row<TC>(lane, r)) * rs + 16 * nt + acc_col(lane)] = acc[mt][nt][r];
        }
}

// MODE 0: plain transform.  MODE 1 (z axis): forward transform, division by
// lambda + nu (Lx_i + Ly_j + Lz_k), backward transform.
//
// Staging: thread t takes the element-local offsets o = t, t + 256, ...
// (consecutive threads read consecutive addresses) and the same offsets of
// every element of the bundle, so the index arithmetic (o -> row within the
// element, column) is done once per offset, not once per value.
template <int AXIS, int NTC, int MT, int MODE, typename TI, typename TO, typename TC>
__global__ void __launch_bounds__(256) k_fdm_axis(FdmArgs A)
{
    constexpr int NB = 16 * NTC;  // columns per work-group; rows: 4 waves x MT tiles of 16
    extern __shared__ __align__(16) unsigned char lds_raw[];
    TC *Bs = (TC *)lds_raw;
    if (A.sc && A.sc->done) return;
    const int bundle = blockIdx.x / A.nchunk;
    const int chunk = blockIdx.x - bundle * A.nchunk;
    const int f0 = chunk * NB;
    const int ncol = min(NB, A.F - f0);
    const int n = A.n, n3 = n * n * n, rs = A.rs, L = A.L, nd = A.nd;
    size_t base, se;
    int i0, i1;
    bundle_base<AXIS>(A, bundle, base, se, i0, i1);
    const double mr = (A.sub_mean && A.sc) ? A.sc->mean_r : 0.0;

    // zero what the products read but the bundle does not fill: rows L..Lp-1
    // and the columns past the chunk's last one
    for (int i = L * rs + threadIdx.x; i < A.Lp * rs; i += blockDim.x) Bs[i] = 0;
    if (ncol < NB)
        for (int i = threadIdx.x; i < L * (NB - ncol); i += blockDim.x) {
            const int k = i / (NB - ncol);
            Bs[k * rs + ncol + (i - k * (NB - ncol))] = 0;
        }
    const TI *in = (const TI *)A.in;
    for (int o = threadIdx.x; o < n3; o += blockDim.x) {
        int ga, f;
        split_o<AXIS>(o, n, ga, f);
        const int c = f - f0;
        if (c < 0 || c >= ncol) continue;
        const TI *src = in + base + o;
        TC *dst = Bs + ga * rs + c;
        for (int e = 0; e < nd; ++e) dst[e * n * rs] = (TC)((double)src[e * se] - mr);
    }
    __syncthreads();

    acc4<TC> acc[MT][NTC];
    gemm_bundle<NTC, MT, TC>((const TC *)A.G, Bs, rs, A.Lp, acc);
    __syncthreads();  // every wave is done reading the bundle
    acc_to_lds<NTC, MT, TC>(acc, Bs, rs, A.Lp);
    __syncthreads();

    if (MODE == 1) {
        // divide by the eigenvalue sums: column c -> (a, b) -> x and y
        // indices, row -> z index
        constexpr int RSTEP = 256 / NB;
        const int c = threadIdx.x % NB, k0 = threadIdx.x / NB;
        if (c < ncol) {
            const int f = f0 + c, b = f / n, a = f - b * n;
            const int gx = i0 * n + a, gy = i1 * n + b;
            const double cxy = A.lambda + A.nu * (A.lam[0][gx] + A.lam[1][gy]);
            const bool zero_col = A.singular && gx == 0 && gy == 0;
            for (int k = k0; k < L; k += RSTEP) {
                const double den = cxy + A.nu * A.lam[2][k];
                Bs[k * rs + c] = (zero_col && k == 0) ? (TC)0 : (TC)((double)Bs[k * rs + c] / den);
            }
        }
        __syncthreads();
        gemm_bundle<NTC, MT, TC>((const TC *)A.G2, Bs, rs, A.Lp, acc);
        __syncthreads();
        acc_to_lds<NTC, MT, TC>(acc, Bs, rs, A.Lp);
        __syncthreads();
    }

    TO *out = (TO *)A.out;
    for (int o = threadIdx.x; o < n3; o += blockDim.x) {
        int ga, f;
        split_o<AXIS>(o, n, ga, f);
        const int c = f - f0;
        if (c < 0 || c >= ncol) continue;
        TO *dst = out + base + o;
        const TC *src = Bs + ga * rs + c;
        for (int e = 0; e < nd; ++e) dst[e * se] = (TO)src[e * n * rs];
    }
}

// a work-group of NTC column tiles covers Lp rows (4 waves x 16/NTC row
// tiles) and its bundle fits the 160 KB of LDS
// LDS row stride of a bundle of NTC column tiles: 16 doubles of padding put
// consecutive rows half the 64 banks apart, so the 4 rows of a B fragment
// read take the minimum two passes
// (one column tile takes 32 doubles of padding: 16 would put every row on
// the same banks)
int lds_stride(int ntc) { return ntc == 1 ? 48 : 16 * ntc + 16; }
int row_tiles(int Lp) { return (Lp / 16 + 3) / 4; }  // per wave
bool ntc_valid(int ntc, int Lp)
{
    if (ntc != 1 && ntc != 2 && ntc != 4) return false;
    const int lds = Lp * lds_stride(ntc) * (int)sizeof(double);
    return row_tiles(Lp) <= 16 / ntc && lds <= 160 * 1024;
}

template <int AXIS, int MODE, typename TI = double, typename TO = double, typename TC = double>
int launch_axis(const MeshDev &m, const FdmDev &f, FdmArgs a, int ntc, hipStream_t s)
{
    const FdmDevAxis &ax = f.ax[AXIS];
    const int n = m.P + 1;
    a.n = n;
    a.nd = m.n[AXIS];
    a.L = ax.L;
    a.Lp = ax.Lp;
    a.nx = m.n[0];
    a.ny = m.n[1];
    a.nz = m.n[2];
    a.F = n * n;
    a.NBc = ntc * 16;
    if (!ntc_valid(ntc, ax.Lp)) {
        set_error("fast diagonalisation: tile shape does not fit this mesh line");
        return DG_ERR_ARG;
    }
    a.nchunk = (a.F + a.NBc - 1) / a.NBc;
    a.rs = lds_stride(ntc);
    const int nbundle = (int)(m.nel / m.n[AXIS]);
    const size_t lds = (size_t)a.Lp * a.rs * sizeof(TC);
    const dim3 grid((unsigned)(nbundle * a.nchunk)), block(256);
    const int mt = row_tiles(ax.Lp);
    auto go = [&](auto NT, auto MTc) {
        hipLaunchKernelGGL((k_fdm_axis<AXIS, decltype(NT)::value, decltype(MTc)::value, MODE, TI, TO, TC>), grid,
                           block, lds, s, a);
    };
    using std::integral_constant;
    if (ntc == 4) {
        switch (mt) {
            case 1: go(integral_constant<int, 4>{}, integral_constant<int, 1>{}); break;
            case 2: go(integral_constant<int, 4>{}, integral_constant<int, 2>{}); break;
            case 3: go(integral_constant<int, 4>{}, integral_constant<int, 3>{}); break;
            default: go(integral_constant<int, 4>{}, integral_constant<int, 4>{}); break;
        }
    } else if (ntc == 1) {
        switch (mt) {
            case 1: go(integral_constant<int, 1>{}, integral_constant<int, 1>{}); break;
            case 2: go(integral_constant<int, 1>{}, integral_constant<int, 2>{}); break;
            case 3: go(integral_constant<int, 1>{}, integral_constant<int, 3>{}); break;
            case 4: go(integral_constant<int, 1>{}, integral_constant<int, 4>{}); break;
            case 5: go(integral_constant<int, 1>{}, integral_constant<int, 5>{}); break;
            case 6: go(integral_constant<int, 1>{}, integral_constant<int, 6>{}); break;
            case 7: go(integral_constant<int, 1>{}, integral_constant<int, 7>{}); break;
            default: go(integral_constant<int, 1>{}, integral_constant<int, 8>{}); break;
        }
    } else {
        switch (mt) {
            case 1: go(integral_constant<int, 2>{}, integral_constant<int, 1>{}); break;
            case 2: go(integral_constant<int, 2>{}, integral_constant<int, 2>{}); break;
            case 3: go(integral_constant<int, 2>{}, integral_constant<int, 3>{}); break;
            case 4: go(integral_constant<int, 2>{}, integral_constant<int, 4>{}); break;
            case 5: go(integral_constant<int, 2>{}, integral_constant<int, 5>{}); break;
            case 6: go(integral_constant<int, 2>{}, integral_constant<int, 6>{}); break;
            case 7: go(integral_constant<int, 2>{}, integral_constant<int, 7>{}); break;
            default: go(integral_constant<int, 2>{}, integral_constant<int, 8>{}); break;
        }
    }
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

// ---- tile-shape autotuner ------------------------------------------------
//
// The column tiles per work-group (NTC = 1, 2 or 4: 16, 32 or 64 mesh lines)
// trade the reuse of each transform matrix fragment read from L2 (more
// columns) against LDS per work-group and the padding of the last chunk of
// a bundle ((P+1)^2 columns per bundle).  Which is fastest depends on the
// degree and the line lengths, so every transform kernel of a new
// (architecture, P, nx, ny, nz) is timed once with each valid NTC on the
// actual data, and the choice is kept in memory and in a cache file (one
// line per mesh shape: "fdm <arch> <P> <nx> <ny> <nz> <ntc_x> <ntc_y> <ntc_z>"),
// $DG_TUNE_CACHE or ~/.cache/dg_sipdg_tune.txt.

std::mutex g_tune_mu;
std::map<std::string, std::array<int, 3>> g_tune;
bool g_tune_loaded = false;

std::string tune_path()
{
    if (const char *e = std::getenv("DG_TUNE_CACHE")) return e;
    const char *h = std::getenv("HOME");
    return h ? std::string(h) + "/.cache/dg_sipdg_tune.txt" : std::string();
}

void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const std::string path = tune_path();
    if (path.empty()) return;
    std::ifstream in(path);
    std::string kind, arch;
    int P, nx, ny, nz, a, b, c;
    while (in >> kind >> arch >> P >> nx >> ny >> nz >> a >> b >> c)
        if (kind == "fdm") {
            char key[160];
            std::snprintf(key, sizeof key, "%s %d %d %d %d", arch.c_str(), P, nx, ny, nz);
            g_tune[key] = {a, b, c};
        }
}

void tune_store(const std::string &key, const std::array<int, 3> &v)
{
    const std::string path = tune_path();
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {  // ~/.cache may not exist yet
        const std::string dir = path.substr(0, slash);
        (void)mkdir(dir.c_str(), 0755);
    }
    std::ofstream out(path, std::ios::app);
    if (out) out << "fdm " << key << " " << v[0] << " " << v[1] << " " << v[2] << "\n";
}

// architecture name of the current device, looked up once per device
// (hipGetDeviceProperties costs about a millisecond: far too much per call)
std::string device_arch()
{
    static std::mutex mu;
    static std::map<int, std::string> names;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    std::lock_guard<std::mutex> lk(mu);
    auto it = names.find(dev);
    if (it != names.end()) return it->second;
    hipDeviceProp_t prop;
    std::string a = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) a = prop.gcnArchName;
    for (char &ch : a)
        if (ch == ' ') ch = '_';
    names[dev] = a;
    return a;
}

// the best of three timed pairs of launches after a warm one (a single pair
// chose the slower shape now and then)
template <int AXIS, int MODE>
int time_axis(const MeshDev &m, const FdmDev &f, FdmArgs a, int ntc, hipStream_t s, hipEvent_t e0,
              hipEvent_t e1, float &ms)
{
    int rc = launch_axis<AXIS, MODE>(m, f, a, ntc, s);  // warm
    if (rc) return rc;
    ms = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
        DG_HIP_CHECK(hipEventRecord(e0, s));
        for (int k = 0; k < 2; ++k)
            if ((rc = launch_axis<AXIS, MODE>(m, f, a, ntc, s))) return rc;
        DG_HIP_CHECK(hipEventRecord(e1, s));
        DG_HIP_CHECK(hipEventSynchronize(e1));
        float t = 0.f;
        DG_HIP_CHECK(hipEventElapsedTime(&t, e0, e1));
        ms = std::min(ms, t);
    }
    return DG_OK;
}

// the NTC of the x, y and z transform kernels for this mesh (tuned at first
// use); in / out: any two distinct vectors of ndof doubles (out is written)
int tile_choice(const MeshDev &m, const FdmDev &f, const FdmArgs &base, const double *in, double *out,
                hipStream_t s, std::array<int, 3> &ntc)
{
    char key[160];
    std::snprintf(key, sizeof key, "%s %d %d %d %d", device_arch().c_str(), m.P, m.n[0], m.n[1], m.n[2]);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            bool ok = true;
            for (int d = 0; d < 3; ++d) ok = ok && ntc_valid(it->second[d], f.ax[d].Lp);
            if (ok) {
                ntc = it->second;
                return DG_OK;
            }
        }
    }
    hipEvent_t e0, e1;
    DG_HIP_CHECK(hipEventCreate(&e0));
    DG_HIP_CHECK(hipEventCreate(&e1));
    FdmArgs a = base;
    a.sc = nullptr;  // time the work itself, never a finished solve's early exit
    a.sub_mean = 0;
    a.in = in;
    a.out = out;
    int rc = DG_OK;
    for (int d = 0; d < 3 && rc == DG_OK; ++d) {
        float best = 1e30f;
        ntc[d] = 0;
        for (int c : {4, 2, 1}) {
            if (!ntc_valid(c, f.ax[d].Lp)) continue;
            float ms = 0.f;
            a.G = f.ax[d].Gf;
            a.G2 = f.ax[d].Gb;
            rc = d == 0 ? time_axis<0, 0>(m, f, a, c, s, e0, e1, ms)
                 : d == 1 ? time_axis<1, 0>(m, f, a, c, s, e0, e1, ms)
                          : time_axis<2, 1>(m, f, a, c, s, e0, e1, ms);
            if (rc == DG_ERR_DEVICE && hipStreamSynchronize(s) == hipSuccess) {
                // this shape could not be launched here (a resource limit):
                // not a candidate
                (void)hipGetLastError();
                rc = DG_OK;
                continue;
            }
            if (rc) break;
            if (ms < best) {
                best = ms;
                ntc[d] = c;
            }
        }
        if (rc == DG_OK && ntc[d] == 0) {
            set_error("fast diagonalisation: no transform tile shape fits this mesh line");
            rc = DG_ERR_ARG;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_tune.emplace(key, ntc).second) tune_store(key, ntc);
    return DG_OK;
}

// per-work-group min and max of a nodal field (grid-stride; up to
// kRangeMaxBlocks work-groups, as many as the partial buffer holds)
constexpr int kRangeMaxBlocks = 1024;
__global__ void __launch_bounds__(256) k_range(const double *__restrict__ v, size_t N, double *partial)
{
    __shared__ double smin[4], smax[4];
    double lo = INFINITY, hi = -INFINITY;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x) {
        const double x = v[i];
        lo = fmin(lo, x);
        hi = fmax(hi, x);
        if (x != x) lo = hi = x;  // a NaN is reported, not skipped
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double ol = __shfl_down(lo, off, 64), oh = __shfl_down(hi, off, 64);
        lo = (ol != ol || lo != lo) ? (lo != lo ? lo : ol) : fmin(lo, ol);
        hi = (oh != oh || hi != hi) ? (hi != hi ? hi : oh) : fmax(hi, oh);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        smin[wid] = lo;
        smax[wid] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
            lo = (smin[k] != smin[k]) ? smin[k] : (lo != lo ? lo : fmin(lo, smin[k]));
            hi = (smax[k] != smax[k]) ? smax[k] : (hi != hi ? hi : fmax(hi, smax[k]));
        }
        partial[blockIdx.x] = lo;
        partial[gridDim.x + blockIdx.x] = hi;
    }
}

}  // namespace

int field_range(const double *v, size_t N, double *partial_dev, size_t partial_cap, double &lo, double &hi,
                hipStream_t s)
{
    const size_t want = std::min<size_t>((N + 255) / 256, (size_t)kRangeMaxBlocks);
    const int nb = (int)std::max<size_t>(1, std::min(want, partial_cap / 2));
    hipLaunchKernelGGL(k_range, dim3(nb), dim3(256), 0, s, v, N, partial_dev);
    DG_HIP_CHECK(hipGetLastError());
    std::vector<double> h(2 * (size_t)nb);
    DG_HIP_CHECK(hipMemcpyAsync(h.data(), partial_dev, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    DG_HIP_CHECK(hipStreamSynchronize(s));
    lo = h[0];
    hi = h[nb];
    bool nan = false;
    for (int k = 0; k < nb; ++k) {
        lo = std::fmin(lo, h[k]);
        hi = std::fmax(hi, h[nb + k]);
        if (h[k] != h[k] || h[nb + k] != h[nb + k]) nan = true;
    }
    if (nan) lo = hi = NAN;
    return DG_OK;
}

size_t fdm_table_bytes(const int n[3], int P)
{
    size_t b = 0;
    for (int d = 0; d < 3; ++d)
        if (n[d] * (P + 1) > kFdmMaxL) return 0;  // no fast diagonalisation on this mesh
    for (int d = 0; d < 3; ++d) {
        const size_t Lp = (size_t)fdm_pad(n[d] * (P + 1));
        b += (2 * Lp * Lp + Lp) * sizeof(double) + 2 * Lp * Lp * sizeof(float);
    }
    return b;
}

int fdm_build_tables(const MeshDev &m, const int bc[3], std::vector<double> &img)
{
    img.assign(fdm_table_bytes(m.n, m.P) / sizeof(double), 0.0);
    size_t off = 0;
    for (int d = 0; d < 3; ++d) {
        int rc = DG_OK;
        const std::shared_ptr<const FdmAxis> ax = fdm_axis_cached(m.v[d], m.P, bc[d], &rc);
        if (!ax) return rc ? rc : DG_ERR_DEVICE;
        const int L = ax->L, Lp = fdm_pad(L);
        double *gf = img.data() + off, *gb = gf + (size_t)Lp * Lp, *lam = gb + (size_t)Lp * Lp;
        for (int k = 0; k < L; ++k)
            for (int i = 0; i < L; ++i) {
                gf[(size_t)k * Lp + i] = ax->S[(size_t)k * L + i];
                gb[(size_t)k * Lp + i] = ax->S[(size_t)i * L + k];
            }
        for (int i = 0; i < L; ++i) lam[i] = ax->lam[i];
        for (int i = L; i < Lp; ++i) lam[i] = 1.0;  // padding rows are never read
        off += 2 * (size_t)Lp * Lp + Lp;
    }
    // the FP32 copies of the matrices, after the FP64 tables of all axes
    float *f32 = (float *)(img.data() + off);
    off = 0;
    for (int d = 0; d < 3; ++d) {
        const int L = m.n[d] * (m.P + 1), Lp = fdm_pad(L);
        const double *gf = img.data() + off;
        for (size_t i = 0; i < 2 * (size_t)Lp * Lp; ++i) f32[i] = (float)gf[i];
        f32 += 2 * (size_t)Lp * Lp;
        off += 2 * (size_t)Lp * Lp + Lp;
    }
    return DG_OK;
}

void fdm_bind(const int n[3], int P, const double *dev, FdmDev &f)
{
    size_t off = 0;
    for (int d = 0; d < 3; ++d) {
        const int L = n[d] * (P + 1), Lp = fdm_pad(L);
        f.ax[d].L = L;
        f.ax[d].Lp = Lp;
        f.ax[d].Gf = dev + off;
        f.ax[d].Gb = dev + off + (size_t)Lp * Lp;
        f.ax[d].lam = dev + off + 2 * (size_t)Lp * Lp;
        off += 2 * (size_t)Lp * Lp + Lp;
    }
    const float *f32 = (const float *)(dev + off);
    for (int d = 0; d < 3; ++d) {
        const size_t Lp = (size_t)f.ax[d].Lp;
        f.ax[d].Gf32 = f32;
        f.ax[d].Gb32 = f32 + Lp * Lp;
        f32 += 2 * Lp * Lp;
    }
}

int fdm_apply(const MeshDev &m, const FdmDev &f, double lambda, double nu, bool singular,
              const double *r, double *z, double *tmp, const void *sc, hipStream_t s)
{
    for (int d = 0; d < 3; ++d)
        if (f.ax[d].L > kFdmMaxL) {
            set_error("fast diagonalisation: a mesh line has more than 512 nodes");
            return DG_ERR_ARG;
        }
    FdmArgs a{};
    a.lam[0] = f.ax[0].lam;
    a.lam[1] = f.ax[1].lam;
    a.lam[2] = f.ax[2].lam;
    a.lambda = lambda;
    a.nu = nu;
    a.sc = (const CgScalars *)sc;
    a.singular = singular ? 1 : 0;
    std::array<int, 3> ntc;
    int rc = tile_choice(m, f, a, r, z, s, ntc);
    if (rc) return rc;
    // forward x (r - mean_r -> z), forward y (z -> tmp), z forward + scale +
    // backward (tmp -> z), backward y (z -> tmp), backward x (tmp -> z)
    a.in = r;
    a.out = z;
    a.G = f.ax[0].Gf;
    a.sub_mean = singular ? 1 : 0;
    if ((rc = launch_axis<0, 0>(m, f, a, ntc[0], s))) return rc;
    a.sub_mean = 0;
    a.in = z;
    a.out = tmp;
    a.G = f.ax[1].Gf;
    if ((rc = launch_axis<1, 0>(m, f, a, ntc[1], s))) return rc;
    a.in = tmp;
    a.out = z;
    a.G = f.ax[2].Gf;
    a.G2 = f.ax[2].Gb;
    if ((rc = launch_axis<2, 1>(m, f, a, ntc[2], s))) return rc;
    a.in = z;
    a.out = tmp;
    a.G = f.ax[1].Gb;
    if ((rc = launch_axis<1, 0>(m, f, a, ntc[1], s))) return rc;
    a.in = tmp;
    a.out = z;
    a.G = f.ax[0].Gb;
    return launch_axis<0, 0>(m, f, a, ntc[0], s);
}

int fdm_apply32(const MeshDev &m, const FdmDev &f, double lambda, double nu, bool singular,
                const double *r, double *z, float *tmp, const void *sc, hipStream_t s)
{
    for (int d = 0; d < 3; ++d)
        if (f.ax[d].L > kFdmMaxL) {
            set_error("fast diagonalisation: a mesh line has more than 512 nodes");
            return DG_ERR_ARG;
        }
    FdmArgs a{};
    a.lam[0] = f.ax[0].lam;
    a.lam[1] = f.ax[1].lam;
    a.lam[2] = f.ax[2].lam;
    a.lambda = lambda;
    a.nu = nu;
    a.sc = (const CgScalars *)sc;
    a.singular = singular ? 1 : 0;
    std::array<int, 3> ntc;  // the tile shapes tuned for the FP64 kernels
    int rc = tile_choice(m, f, a, r, z, s, ntc);
    if (rc) return rc;
    float *t0 = tmp, *t1 = tmp + m.ndof;
    // forward x (r - mean_r -> t0, to FP32), forward y (t0 -> t1), z forward +
    // scale + backward (t1 -> t0), backward y (t0 -> t1), backward x (t1 -> z,
    // to FP64)
    a.in = r;
    a.out = t0;
    a.G = f.ax[0].Gf32;
    a.sub_mean = singular ? 1 : 0;
    if ((rc = launch_axis<0, 0, double, float, float>(m, f, a, ntc[0], s))) return rc;
    a.sub_mean = 0;
    a.in = t0;
    a.out = t1;
    a.G = f.ax[1].Gf32;
    if ((rc = launch_axis<1, 0, float, float, float>(m, f, a, ntc[1], s))) return rc;
    a.in = t1;
    a.out = t0;
    a.G = f.ax[2].Gf32;
    a.G2 = f.ax[2].Gb32;
    if ((rc = launch_axis<2, 1, float, float, float>(m, f, a, ntc[2], s))) return rc;
    a.in = t0;
    a.out = t1;
    a.G = f.ax[1].Gb32;
    if ((rc = launch_axis<1, 0, float, float, float>(m, f, a, ntc[1], s))) return rc;
    a.in = t1;
    a.out = z;
    a.G = f.ax[0].Gb32;
    return launch_axis<0, 0, float, double, float>(m, f, a, ntc[0], s);
}

}  // namespace dg
