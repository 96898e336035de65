// Fast-diagonalisation preconditioner (internal): the exact inverse of the
// constant-nu SIP-DG operator on a Cartesian product mesh, applied by three
// dense 1D transforms per direction (MFMA contractions along the mesh axes).
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <vector>

#include "dg_internal.h"

namespace dg {

// Generalised eigendecomposition of one axis: K S = M S diag(lam),
// S^T M S = I.  S is L x L, row-major (S[g][j]: node g, mode j), L = n_d (P+1).
struct FdmAxis {
    int L = 0;
    std::vector<double> lam;
    std::vector<double> S;
};

// symmetric eigenproblem A V = V diag(lam), eigenvalues ascending
bool sym_eig(int n, std::vector<double> A, std::vector<double> &lam, std::vector<double> &V);
int fdm_axis_compute(const std::vector<double> &v, int P, int bc, FdmAxis &out);
std::shared_ptr<const FdmAxis> fdm_axis_cached(const std::vector<double> &v, int P, int bc, int *rc);

constexpr int kFdmMaxL = 512;  // longest mesh line (n_d (P+1)) the kernels take

// Device tables of one axis: the forward and backward contraction matrices,
// padded to Lp = L rounded up to 16, stored [k][i'] (input row k, output row
// i') as the kernels read them, and the eigenvalues; FP32 copies of the
// matrices follow the FP64 tables of all three axes.
struct FdmDevAxis {
    int L = 0, Lp = 0;
    const double *Gf = nullptr;   // Gf[k][i'] = S[k][i']   (t = S^T r)
    const double *Gb = nullptr;   // Gb[k][i'] = S[i'][k]   (z = S t)
    const double *lam = nullptr;  // Lp values
    const float *Gf32 = nullptr;  // FP32 copies of Gf and Gb
    const float *Gb32 = nullptr;
};

struct FdmDev {
    FdmDevAxis ax[3];
};

inline int fdm_pad(int L) { return (L + 15) & ~15; }
// bytes of the device tables of a mesh (all three axes)
size_t fdm_table_bytes(const int n[3], int P);
// host image of the tables for the given BCs, in the layout fdm_bind expects
int fdm_build_tables(const MeshDev &m, const int bc[3], std::vector<double> &img);
// pointers into a device copy of that image
void fdm_bind(const int n[3], int P, const double *dev, FdmDev &f);

// z = (S (x) S (x) S) (lambda + nu Lam)^-1 (S (x) S (x) S)^T (r - mean_r)
// (mean_r from sc when singular; the zero mode dropped when singular).
// tmp: one scratch vector of ndof doubles.  Every kernel returns at once
// when sc->done is set (sc may be null: always run).
int fdm_apply(const MeshDev &m, const FdmDev &f, double lambda, double nu, bool singular,
              const double *r, double *z, double *tmp, const void *sc, hipStream_t s);
// The same with FP32 transforms (FP32 matrices, MFMA arithmetic and
// intermediates; r read and z written in FP64): the FP32 preconditioner.
// tmp: 2 ndof floats of scratch.
int fdm_apply32(const MeshDev &m, const FdmDev &f, double lambda, double nu, bool singular,
                const double *r, double *z, float *tmp, const void *sc, hipStream_t s);

// min and max of a device field of N values (NaN if any is NaN); partial_dev
// holds partial_cap >= 2 doubles (one min and one max per work-group);
// synchronises the stream
int field_range(const double *v, size_t N, double *partial_dev, size_t partial_cap, double &lo, double &hi,
                hipStream_t s);

}  // namespace dg
