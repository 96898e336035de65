// Request server: continuous batching of implicit-stage solves.
//
// Requests (Helmholtz or pressure Poisson solves on n^3-element periodic
// cubes of degree P, Alg. 3 of arXiv 2112.04167) arrive at any time.  The
// server owns one device arena of the configured HBM budget.  A scheduler
// thread admits requests in arrival order as soon as a slot is free and the
// request's footprint (geometry, right-hand side, solution, solver
// workspace) can be carved from the arena; each slot is a host thread with
// its own HIP stream that runs the solve there, so solves admitted at
// different times overlap on the device.  Completion frees the request's
// memory (the solution too unless it is kept for fetching), which lets the
// scheduler admit the next request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "dg_internal.h"
#include "fdm.h"
#include "kernels.h"

namespace dg {

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// f_i = 2 u_i - 1, u_i = (z_i >> 11) 2^-53 with z_i the (i+1)-th output of
// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) started from `seed`.
__global__ void k_splitmix_uniform(double *f, size_t n, unsigned long long seed)
{
    const unsigned long long gamma = 0x9E3779B97F4A7C15ull;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        unsigned long long z = seed + (unsigned long long)(i + 1) * gamma;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        f[i] = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
    }
}

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) of the device arena.
class Arena {
public:
    void init(size_t size) { free_[0] = size; size_ = size; }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = al256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = al256(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0;
};

struct Req {
    int64_t id;
    dg_request d;
    std::vector<double> rhs;  // host copy (when given)
    int64_t ndof;
    size_t work_bytes, x_bytes, geo_bytes, ws_bytes;
    size_t work_off = 0, x_off = 0;
    double t_submit = 0, t_start = 0, t_done = 0;
    int state = 0;  // 0 queued, 1 running, 2 done
    int status = DG_PENDING;
    dg_solve_info info{};
    bool x_held = false;
};

}  // namespace

class Server {
public:
    Server(size_t budget, int slots) : budget_(budget), nslots_(slots) {}

    int start()
    {
        hipError_t e = hipMalloc(&arena_base_, budget_);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error("server arena allocation failed");
            return DG_ERR_OOM;
        }
        arena_.init(budget_);
        DG_HIP_CHECK(hipStreamCreateWithFlags(&io_stream_, hipStreamNonBlocking));
        slot_.reset(new Slot[nslots_]);
        for (int k = 0; k < nslots_; ++k) {
            DG_HIP_CHECK(hipStreamCreateWithFlags(&slot_[k].stream, hipStreamNonBlocking));
            DG_HIP_CHECK(hipHostMalloc(&slot_[k].host_sc, solve_host_scalar_bytes(), 0));
        }
        DG_HIP_CHECK(hipGetDevice(&device_));
        for (int k = 0; k < nslots_; ++k) slot_[k].th = std::thread([this, k] { slot_loop(k); });
        sched_ = std::thread([this] { sched_loop(); });
        return DG_OK;
    }

    ~Server()
    {
        {
            std::unique_lock<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        if (slot_)
            for (int k = 0; k < nslots_; ++k) slot_[k].cv.notify_all();
        if (sched_.joinable()) sched_.join();
        if (slot_) {
            for (int k = 0; k < nslots_; ++k)
                if (slot_[k].th.joinable()) slot_[k].th.join();
            for (int k = 0; k < nslots_; ++k) {
                if (slot_[k].stream) (void)hipStreamDestroy(slot_[k].stream);
                if (slot_[k].host_sc) (void)hipHostFree(slot_[k].host_sc);
            }
        }
        if (io_stream_) (void)hipStreamDestroy(io_stream_);
        if (arena_base_) (void)hipFree(arena_base_);
    }

    int submit(const dg_request *r, int64_t *id)
    {
        if (!r || !id || r->n < 1 || r->P < kMinPKernel || r->P > kMaxPKernel || !(r->tol > 0.0) ||
            (r->precision != DG_FP64 && r->precision != DG_MIXED) ||
            (r->precond != DG_PC_JACOBI && r->precond != DG_PC_FDM) ||
            (r->precond == DG_PC_FDM && (r->precision != DG_FP64 || r->n * (r->P + 1) > kFdmMaxL)) ||
            (!r->is_poisson && !(r->lambda > 0.0 && std::isfinite(r->lambda)))) {
            set_error("bad request");
            return DG_ERR_ARG;
        }
        const int n3[3] = {r->n, r->n, r->n};
        const int64_t nd = (int64_t)r->n * r->n * r->n * (r->P + 1) * (r->P + 1) * (r->P + 1);
        if (nd >= (int64_t)1 << 31) {
            set_error("request mesh too large");
            return DG_ERR_ARG;
        }
        auto q = std::make_unique<Req>();
        q->d = *r;
        q->ndof = nd;
        q->geo_bytes = al256(mesh_geo_bytes(n3, r->P));
        q->ws_bytes = al256(solve_footprint_for(n3, r->P, r->precision));
        q->x_bytes = al256((size_t)nd * sizeof(double));
        q->work_bytes = q->geo_bytes + q->ws_bytes + al256((size_t)nd * sizeof(double));
        if (q->work_bytes + q->x_bytes > budget_) {
            set_error("request footprint exceeds the server budget");
            return DG_ERR_BUDGET;
        }
        if (r->rhs) q->rhs.assign(r->rhs, r->rhs + nd);
        q->d.rhs = nullptr;
        std::unique_lock<std::mutex> lk(mu_);
        q->id = next_id_++;
        q->t_submit = now_s();
        if (first_submit_ < 0) first_submit_ = q->t_submit;
        *id = q->id;
        queue_.push_back(q.get());
        reqs_[q->id] = std::move(q);
        ++outstanding_;
        lk.unlock();
        cv_.notify_all();
        return DG_OK;
    }

    int poll(int64_t id, dg_solve_info *info)
    {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(id);
        if (it == reqs_.end()) {
            set_error("unknown request id");
            return DG_ERR_ARG;
        }
        Req *q = it->second.get();
        if (q->state != 2) return DG_PENDING;
        if (info) *info = q->info;
        return q->status;
    }

    int fetch(int64_t id, double *x)
    {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(id);
        if (it == reqs_.end() || !x) {
            set_error("unknown request id or null output");
            return DG_ERR_ARG;
        }
        Req *q = it->second.get();
        if (q->state != 2) return DG_PENDING;
        if (!q->x_held) {
            set_error("result not kept (keep_result = 0) or already fetched");
            return DG_ERR_ARG;
        }
        const size_t off = q->x_off;
        const int64_t nd = q->ndof;
        q->x_held = false;  // a second fetch of the same result is refused
        ++fetching_;
        lk.unlock();
        hipError_t e = hipMemcpyAsync(x, (char *)arena_base_ + off, (size_t)nd * sizeof(double),
                                      hipMemcpyDeviceToHost, io_stream_);
        if (e == hipSuccess) e = hipStreamSynchronize(io_stream_);
        lk.lock();
        arena_.release(q->x_off, q->x_bytes);
        --fetching_;
        lk.unlock();
        cv_.notify_all();
        if (e != hipSuccess) {
            set_error(std::string("result copy failed: ") + hipGetErrorString(e));
            return DG_ERR_DEVICE;
        }
        return DG_OK;
    }

    int drain()
    {
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [this] { return outstanding_ == 0; });
        return DG_OK;
    }

    int stats(dg_server_stats *st)
    {
        std::unique_lock<std::mutex> lk(mu_);
        std::vector<double> lat;
        double last = -1;
        for (auto &kv : reqs_) {
            const Req *q = kv.second.get();
            if (q->state != 2) continue;
            lat.push_back(q->t_done - q->t_submit);
            last = std::max(last, q->t_done);
        }
        std::memset(st, 0, sizeof(*st));
        st->completed = (int64_t)lat.size();
        st->peak_bytes = (double)peak_bytes_;
        st->peak_active = peak_active_;
        if (lat.empty()) return DG_OK;
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double p) {  // nearest rank
            size_t k = (size_t)std::ceil(p * lat.size());
            k = std::max<size_t>(1, std::min(k, lat.size()));
            return lat[k - 1];
        };
        st->p50 = pct(0.50);
        st->p99 = pct(0.99);
        double s = 0;
        for (double v : lat) s += v;
        st->mean = s / lat.size();
        st->max = lat.back();
        st->makespan = last - first_submit_;
        return DG_OK;
    }

private:
    struct Slot {
        hipStream_t stream = nullptr;
        void *host_sc = nullptr;
        std::thread th;
        std::condition_variable cv;
        Req *job = nullptr;
    };

    void sched_loop()
    {
        (void)hipSetDevice(device_);
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_.wait(lk, [this] { return stop_ || (!queue_.empty() && free_slot() >= 0); });
            if (stop_) return;
            Req *q = queue_.front();
            size_t off_w, off_x;
            bool fits = arena_.alloc(q->work_bytes, off_w);
            if (fits && !arena_.alloc(q->x_bytes, off_x)) {
                arena_.release(off_w, q->work_bytes);
                fits = false;
            }
            if (!fits) {
                // Only a finishing solve or a fetch frees memory.  With neither
                // in progress, the space is held by kept results that nobody is
                // fetching: waiting would never end (and drain() would block
                // for good), so the request fails instead.
                if (active_ == 0 && fetching_ == 0) {
                    queue_.pop_front();
                    q->state = 2;
                    q->status = DG_ERR_BUDGET;
                    q->info = dg_solve_info{};
                    q->info.status = DG_ERR_BUDGET;
                    q->t_start = q->t_done = now_s();
                    q->rhs.clear();
                    q->rhs.shrink_to_fit();
                    --outstanding_;
                    done_cv_.notify_all();
                    continue;
                }
                cv_.wait(lk);  // until memory is released
                continue;
            }
            queue_.pop_front();
            q->work_off = off_w;
            q->x_off = off_x;
            q->x_held = true;
            q->state = 1;
            q->t_start = now_s();
            const int k = free_slot();
            slot_[k].job = q;
            ++active_;
            peak_active_ = std::max(peak_active_, active_);
            peak_bytes_ = std::max(peak_bytes_, arena_.used());
            slot_[k].cv.notify_all();
        }
    }

    int free_slot() const
    {
        for (int k = 0; k < nslots_; ++k)
            if (!slot_[k].job) return k;
        return -1;
    }

    void slot_loop(int k)
    {
        (void)hipSetDevice(device_);
        Slot &S = slot_[k];
        for (;;) {
            Req *q;
            {
                std::unique_lock<std::mutex> lk(mu_);
                S.cv.wait(lk, [&] { return stop_ || S.job != nullptr; });
                if (stop_ && !S.job) return;
                q = S.job;
            }
            dg_solve_info info{};
            const int rc = run(q, S, info);
            {
                std::unique_lock<std::mutex> lk(mu_);
                q->t_done = now_s();
                q->status = rc;
                q->info = info;
                q->info.status = rc;
                q->state = 2;
                arena_.release(q->work_off, q->work_bytes);
                if (!q->d.keep_result) {
                    arena_.release(q->x_off, q->x_bytes);
                    q->x_held = false;
                }
                q->rhs.clear();
                q->rhs.shrink_to_fit();
                S.job = nullptr;
                --active_;
                --outstanding_;
            }
            cv_.notify_all();
            done_cv_.notify_all();
        }
    }

    int run(Req *q, Slot &S, dg_solve_info &info)
    {
        const int n = q->d.n, P = q->d.P;
        std::vector<double> v(n + 1);
        for (int i = 0; i <= n; ++i) v[i] = (double)i / n;
        v[n] = 1.0;
        const int bc[3] = {DG_BC_PERIODIC, DG_BC_PERIODIC, DG_BC_PERIODIC};
        char *base = (char *)arena_base_ + q->work_off;
        void *geo = base;
        void *ws = base + q->geo_bytes;
        double *rhs = (double *)(base + q->geo_bytes + q->ws_bytes);
        double *x = (double *)((char *)arena_base_ + q->x_off);
        dg_mesh *m = nullptr;
        int rc = mesh_create_impl(n, n, n, P, v.data(), v.data(), v.data(), bc, S.stream, geo, &m);
        if (rc) return rc;
        mesh_lend_workspace(m, ws, q->ws_bytes, S.host_sc);
        const size_t N = (size_t)q->ndof;
        if (!q->rhs.empty()) {
            hipError_t e = hipMemcpyAsync(rhs, q->rhs.data(), N * sizeof(double), hipMemcpyHostToDevice,
                                          S.stream);
            if (e != hipSuccess) {
                dg_mesh_destroy(m);
                set_error("rhs upload failed");
                return DG_ERR_DEVICE;
            }
        } else {
            const unsigned blocks = (unsigned)std::min<size_t>((N + 255) / 256, 4096);
            hipLaunchKernelGGL(k_splitmix_uniform, dim3(std::max(1u, blocks)), dim3(256), 0, S.stream,
                               rhs, N, (unsigned long long)q->d.rhs_seed);
        }
        // the solvers start from the given x: start from zero
        if (hipMemsetAsync(x, 0, N * sizeof(double), S.stream) != hipSuccess) {
            dg_mesh_destroy(m);
            set_error("clearing x failed");
            return DG_ERR_DEVICE;
        }
        dg_solve_opts o;
        dg_default_opts(&o);
        o.tol = q->d.tol;
        o.precision = q->d.precision;
        o.precond = q->d.precond;
        if (q->d.is_poisson)
            rc = poisson_solve(m, rhs, x, &o, &info);
        else
            rc = helmholtz_solve(m, q->d.lambda, nullptr, 1.0, rhs, x, &o, &info);
        dg_mesh_destroy(m);
        return rc;
    }

    size_t budget_;
    int nslots_;
    int device_ = 0;
    void *arena_base_ = nullptr;
    Arena arena_;
    hipStream_t io_stream_ = nullptr;
    std::unique_ptr<Slot[]> slot_;
    std::thread sched_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    std::deque<Req *> queue_;
    std::map<int64_t, std::unique_ptr<Req>> reqs_;
    int64_t next_id_ = 0;
    int64_t outstanding_ = 0;
    int active_ = 0, peak_active_ = 0;
    int fetching_ = 0;  // fetches copying a result out (their memory is freed after)
    size_t peak_bytes_ = 0;
    double first_submit_ = -1;
    bool stop_ = false;
};

}  // namespace dg

extern "C" {

int dg_server_create(size_t hbm_budget_bytes, int max_slots, void **srv)
{
    if (!srv || max_slots < 1 || max_slots > 64 || hbm_budget_bytes < (1u << 20)) {
        dg::set_error("need max_slots in 1..64 and a budget of at least 1 MiB");
        return DG_ERR_ARG;
    }
    auto s = std::make_unique<dg::Server>(hbm_budget_bytes, max_slots);
    if (int rc = s->start()) return rc;
    *srv = s.release();
    return DG_OK;
}

int dg_server_submit(void *srv, const dg_request *req, int64_t *req_id)
{
    if (!srv) return DG_ERR_ARG;
    return static_cast<dg::Server *>(srv)->submit(req, req_id);
}

int dg_server_poll(void *srv, int64_t req_id, dg_solve_info *info)
{
    if (!srv) return DG_ERR_ARG;
    return static_cast<dg::Server *>(srv)->poll(req_id, info);
}

int dg_server_fetch(void *srv, int64_t req_id, double *x_host)
{
    if (!srv) return DG_ERR_ARG;
    return static_cast<dg::Server *>(srv)->fetch(req_id, x_host);
}

int dg_server_drain(void *srv)
{
    if (!srv) return DG_ERR_ARG;
    return static_cast<dg::Server *>(srv)->drain();
}

int dg_server_get_stats(void *srv, dg_server_stats *st)
{
    if (!srv || !st) return DG_ERR_ARG;
    return static_cast<dg::Server *>(srv)->stats(st);
}

int dg_server_destroy(void *srv)
{
    if (!srv) return DG_OK;
    auto *s = static_cast<dg::Server *>(srv);
    s->drain();
    delete s;
    return DG_OK;
}

}  // extern "C"
