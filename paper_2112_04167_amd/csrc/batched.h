// Host interface of the persistent batched solver (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "dg_internal.h"

namespace dg {

constexpr int kMaxBatch = 8;
constexpr int kBatchMaxBlocks = 4096;           // resident work-groups at most
constexpr int kBatchNC = 8;                     // reduction components per system and phase
constexpr int kBatchSlots = kBatchNC * kMaxBatch;
constexpr int kBatchHandoff = 3;                // result status: left to the single-system solver

struct BatchSysDesc {
    double *x64, *b64, *r64;            // solution (caller), load, FP64 residual
    const double *rhs, *nu64;           // right-hand side, FP64 nu field or null
    void *xi, *ri, *pi, *qi, *ui, *si, *di;  // inner-precision CG vectors (di = 1/diag)
    const void *nui;                    // inner-precision nu field or null
    double lambda;
    int bc[3];
    int singular;
};

struct BatchRequest {
    int nsys;
    BatchSysDesc sys[kMaxBatch];
    void *results;    // device, batched_result_bytes()
    void *sync;       // device, batched_sync_bytes(); its counters are cleared per launch
    double *partial;  // device, batched_partial_doubles()
    double tol;       // FP64 stopping tolerance (relative, collocation RMS residual)
    double delta;     // replacement threshold on the recurrence residual (0: only at convergence)
    double mass_mean; // domain volume / ndof: typical GLL mass, sets the inner scaling
    int maxit;        // cap on inner iterations (per system)
    int max_replace;  // cap on FP64 residual replacements (per system)
    int weak;
    int handoff;      // end the launch once a single system is left unconverged (its x64
                      // then holds the current solution; result status kBatchHandoff)
    bool inner_fp32;
};

struct BatchSysResult {
    int status, iters, replaced;
    double bnorm2, res64;
};

size_t batched_sync_bytes();
size_t batched_result_bytes();
size_t batched_partial_doubles();
// launches the solve (autotuning the launch shape on first use of a shape key)
int batched_launch(const MeshDev &m, const BatchRequest &req, hipStream_t stream, int *blocks_per_cu);
// after the stream has completed: per-system results and the barrier's error flag
int batched_read_results(const void *host_results, int s, BatchSysResult *out);
int batched_check_sync(const void *host_sync_err);
size_t batched_sync_err_offset();

}  // namespace dg
