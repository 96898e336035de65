// Host interface of the persistent batched solver (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "dg_internal.h"

namespace dg {

constexpr int kMaxBatch = 8;

struct BatchSysDesc {
    double *x64, *b64, *r64;
    const double *rhs, *nu64;
    void *xi, *ri, *pi, *qi, *di, *bi;  // inner-precision vectors
    const void *nui;                    // inner-precision nu field or null
    double lambda;
    int bc[3];
    int singular;
};

struct BatchRequest {
    int nsys;
    BatchSysDesc sys[kMaxBatch];
    void *state;  // device, batched_state_bytes()
    double *partial;
    unsigned *counter;
    double tol, inner_tol;
    int maxit_outer, inner_maxit, weak;
    bool inner_fp32;
};

struct BatchResult {
    int blocks_per_cu;
};

struct BatchSysResult {
    int status, outer, inner_total;
    double bnorm2, res2;
};

// partial-sum slots per resident work-group and parity buffer (two buffers)
constexpr int kBatchPartialPerBlock = 5 * kMaxBatch;
constexpr int kBatchMaxBlocks = 4096;  // resident work-groups at most

int batched_launch(const MeshDev &m, const BatchRequest &req, hipStream_t stream, BatchResult *res);
size_t batched_state_bytes();
int batched_read_state(const void *host_state, int s, BatchSysResult *out);

}  // namespace dg
