// Device-side helpers shared by the HIP kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "dg_internal.h"

namespace dg {

// --------------------------------------------------------------- helpers --

template <int P>
struct Shape {
    static constexpr int n = P + 1;
    static constexpr int NL = n * n;        // lines per element per direction
    static constexpr int N3 = n * n * n;    // nodes per element
    static constexpr int EB = (256 / NL) > 0 ? (256 / NL) : 1;  // elements per group
    static constexpr int NT = EB * NL;      // active threads
    static constexpr int NTP = ((NT + 63) / 64) * 64;            // launched threads
};

__device__ __forceinline__ int xcd_remap(int bid, int nblk)
{
    // blocks are dispatched round-robin over 8 XCDs; give XCD k a contiguous
    // range of logical blocks
    const int q = nblk >> 3, rem = nblk & 7;
    const int xcd = bid & 7, k = bid >> 3;
    return xcd < rem ? xcd * (q + 1) + k : rem * (q + 1) + (xcd - rem) * q + k;
}

template <typename T>
__device__ __forceinline__ T dmax(T a, T b) { return a > b ? a : b; }
template <typename T>
__device__ __forceinline__ T dmin(T a, T b) { return a < b ? a : b; }

// face kind of the low / high end of element index k along an axis
// returns 0 = natural (nothing), 1 = neighbour (interior or periodic), 2 = Dirichlet
__device__ __forceinline__ int face_kind(int k, int nk, int bc, bool high, int &knb)
{
    if (!high) {
        if (k > 0) { knb = k - 1; return 1; }
        if (bc == DG_BC_PERIODIC) { knb = nk - 1; return 1; }
    } else {
        if (k < nk - 1) { knb = k + 1; return 1; }
        if (bc == DG_BC_PERIODIC) { knb = 0; return 1; }
    }
    knb = k;
    return bc == DG_BC_DIRICHLET ? 2 : 0;
}

// wave64 + block reduction of NC doubles; result valid in thread 0
template <int NC>
__device__ __forceinline__ void block_sum(double (&v)[NC], double *sh /* >= 16*NC */)
{
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_down(v[c], off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NC; ++c) sh[c * 16 + wid] = v[c];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double s = 0.0;
            for (int k = 0; k < nw; ++k) s += sh[c * 16 + k];
            v[c] = s;
        }
    }
    __syncthreads();
}

// Write this work-group's sums to partial[c * nblk + blockIdx.x] (plain
// stores: the consumer is a later kernel).
template <int NC>
__device__ __forceinline__ void publish_partials(double (&v)[NC], double *partial, int nblk, double *sh)
{
    block_sum<NC>(v, sh);
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < NC; ++c) partial[(size_t)c * nblk + blockIdx.x] = v[c];
}

}  // namespace dg
