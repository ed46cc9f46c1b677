// Serving engine: continuous batching of many inverse problems on one GPU.
//
// Requests (each with its own data y, noise variances, observation count, chain count
// and step budget) wait in arrival order. Every observation-count bucket owns a pool:
// a problem with a fixed number of chain slots and request rows. A request is
// admitted into the smallest bucket that covers its d_y as soon as its chains fit a
// contiguous free slot range and a request row is free (admission by memory: every
// slot is preallocated HBM). Outputs beyond a request's d_y get Gamma^-1/2 = 0, so
// they drop out of the misfit, the ppg and the GN Hessian.
//
// A pool advances every occupied slot with one batched launch per stage and step
// (run_steps over slots [0, highest occupied + 1)), in quanta of K steps on its own
// stream; pools of different buckets overlap on the device. An admitted request's
// chains join at the next step (fresh: the step draws their prior initial states and
// builds the cache), then take exactly n_steps Markov steps and go idle. Keys are
// per request, so a request's chains draw the same numbers whatever else runs.
//
// When the quantum that contains a request's last step has been enqueued, its
// reduction is enqueued behind it on the same stream: xbar = mean of the post-burn-in
// states over its chains and steps (burn-in: the first 20%), the posterior mean field
// Psi_r xbar, and the acceptance counts, copied to pinned host memory. When that copy
// has completed the request is finished; its slots and row are freed for the next
// admissions.
#include <chrono>
#include <deque>
#include <thread>

#include "dino_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

enum ReqState { REQ_PENDING, REQ_LIVE, REQ_REDUCING, REQ_DONE, REQ_POLLED };

struct Req {
    dino_request spec{};
    std::vector<double> y, winv;
    int state = REQ_PENDING;
    int pool = -1, c0 = -1, row = -1;
    int64_t admit_step = 0, finish_step = 0;
    double admitted = 0.0, finished = 0.0;
    hipEvent_t done_ev = nullptr;
    std::vector<double> mean;
    int64_t accepts = 0, failures = 0;
};

__global__ void count_kernel(int c0, int n, const int64_t* __restrict__ acc, const int64_t* __restrict__ fail,
                             int64_t* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int64_t a = 0, f = 0;
        for (int c = c0; c < c0 + n; ++c) {
            a += acc[c];
            f += fail[c];
        }
        out[0] = a;
        out[1] = f;
    }
}

__global__ void zero_counts_kernel(int c0, int n, int64_t* __restrict__ acc, int64_t* __restrict__ fail) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) {
        acc[c0 + k] = 0;
        fail[c0 + k] = 0;
    }
}

struct Pool {
    int dy = 0;
    dino_problem* p = nullptr;
    hipStream_t stream = nullptr;
    std::vector<int> slot_owner;      // request per slot, -1 free
    std::vector<int> row_owner;       // request per row, -1 free
    int64_t enqueued = 0;             // steps enqueued so far
    std::deque<hipEvent_t> inflight;  // one event per enqueued quantum
    std::vector<hipEvent_t> spare;
    double* d_xbar = nullptr;         // rows x r
    double* d_field = nullptr;        // rows x d_m
    int64_t* d_counts = nullptr;      // rows x 2
    double* h_rows = nullptr;         // pinned: rows x 2 dy (y, winv)
    double* h_field = nullptr;        // pinned: rows x d_m
    int64_t* h_counts = nullptr;      // pinned: rows x 2

    hipEvent_t event() {
        if (!spare.empty()) {
            hipEvent_t e = spare.back();
            spare.pop_back();
            return e;
        }
        hipEvent_t e;
        DINO_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        return e;
    }
};

}  // namespace

struct dino_server {
    dino_ctx* ctx = nullptr;
    dino_server_cfg cfg{};
    Clock::time_point t0;
    std::vector<Pool> pools;
    std::vector<Req> reqs;
    std::deque<int> pending;
    std::deque<int> finished;
    int64_t chain_steps = 0;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

using namespace dino;

namespace {

// First slot of a free contiguous range of n slots, or -1.
int find_slots(const Pool& pl, int n) {
    int run = 0;
    for (int c = 0; c < (int)pl.slot_owner.size(); ++c) {
        run = pl.slot_owner[c] < 0 ? run + 1 : 0;
        if (run == n) return c - n + 1;
    }
    return -1;
}

int find_row(const Pool& pl) {
    for (int k = 0; k < (int)pl.row_owner.size(); ++k)
        if (pl.row_owner[k] < 0) return k;
    return -1;
}

int bucket_of(const dino_server* s, int dy) {
    for (int b = 0; b < (int)s->pools.size(); ++b)
        if (s->pools[b].dy >= dy) return b;
    return -1;
}

void admit(dino_server* s, int id) {
    Req& q = s->reqs[id];
    Pool& pl = s->pools[q.pool];
    dino_problem* p = pl.p;
    const int dy = pl.dy;
    double* hy = pl.h_rows + (size_t)q.row * 2 * dy;
    double* hw = hy + dy;
    for (int i = 0; i < dy; ++i) {
        hy[i] = i < q.spec.d_y ? q.y[i] : 0.0;
        hw[i] = i < q.spec.d_y ? q.winv[i] : 0.0;
    }
    DINO_HIP(hipMemcpyAsync(p->y + (size_t)q.row * dy, hy, sizeof(double) * dy, hipMemcpyHostToDevice, pl.stream));
    DINO_HIP(hipMemcpyAsync(p->winv + (size_t)q.row * dy, hw, sizeof(double) * dy, hipMemcpyHostToDevice,
                            pl.stream));
    const int64_t burn = q.spec.n_steps / 5;
    launch_meta_fill(p, q.c0, q.spec.n_chains, q.spec.seed, q.spec.request_id, q.spec.n_steps, burn, q.row,
                     CHAIN_FRESH, 0, pl.stream);
    hipLaunchKernelGGL(zero_counts_kernel, dim3((q.spec.n_chains + 255) / 256), dim3(256), 0, pl.stream, q.c0,
                       q.spec.n_chains, p->accepts, p->failures);
    DINO_HIP(hipGetLastError());
    for (int c = q.c0; c < q.c0 + q.spec.n_chains; ++c) pl.slot_owner[c] = id;
    pl.row_owner[q.row] = id;
    q.admit_step = pl.enqueued;
    q.finish_step = pl.enqueued + 1 + q.spec.n_steps;  // one fresh step, then n_steps Markov steps
    q.admitted = s->now();
    q.state = REQ_LIVE;
}

void enqueue_reduction(dino_server* s, int id) {
    Req& q = s->reqs[id];
    Pool& pl = s->pools[q.pool];
    dino_problem* p = pl.p;
    const int d_m = s->ctx->basis.d_m;
    const int64_t count = q.spec.n_steps - q.spec.n_steps / 5;
    double* xbar = pl.d_xbar + (size_t)q.row * p->r;
    double* field = pl.d_field + (size_t)q.row * d_m;
    launch_request_mean(p, q.c0, q.spec.n_chains, count, xbar, field, pl.stream);
    hipLaunchKernelGGL(count_kernel, dim3(1), dim3(64), 0, pl.stream, q.c0, q.spec.n_chains, p->accepts,
                       p->failures, pl.d_counts + 2 * q.row);
    DINO_HIP(hipGetLastError());
    DINO_HIP(hipMemcpyAsync(pl.h_field + (size_t)q.row * d_m, field, sizeof(double) * d_m, hipMemcpyDeviceToHost,
                            pl.stream));
    DINO_HIP(hipMemcpyAsync(pl.h_counts + 2 * q.row, pl.d_counts + 2 * q.row, 2 * sizeof(int64_t),
                            hipMemcpyDeviceToHost, pl.stream));
    q.done_ev = pl.event();
    DINO_HIP(hipEventRecord(q.done_ev, pl.stream));
    q.state = REQ_REDUCING;
}

void complete(dino_server* s, int id) {
    Req& q = s->reqs[id];
    Pool& pl = s->pools[q.pool];
    const int d_m = s->ctx->basis.d_m;
    q.finished = s->now();
    q.mean.assign(pl.h_field + (size_t)q.row * d_m, pl.h_field + (size_t)(q.row + 1) * d_m);
    q.accepts = pl.h_counts[2 * q.row];
    q.failures = pl.h_counts[2 * q.row + 1];
    pl.spare.push_back(q.done_ev);
    q.done_ev = nullptr;
    for (int c = q.c0; c < q.c0 + q.spec.n_chains; ++c) pl.slot_owner[c] = -1;
    pl.row_owner[q.row] = -1;
    q.state = REQ_DONE;
    s->chain_steps += (int64_t)q.spec.n_chains * q.spec.n_steps;
    s->finished.push_back(id);
}

// One pass of the scheduler; returns true if it did anything.
bool pass(dino_server* s) {
    bool acted = false;
    const double t = s->now();
    // finished reductions
    for (auto& pl : s->pools) {
        while (!pl.inflight.empty() && hipEventQuery(pl.inflight.front()) == hipSuccess) {
            pl.spare.push_back(pl.inflight.front());
            pl.inflight.pop_front();
        }
    }
    for (size_t id = 0; id < s->reqs.size(); ++id) {
        Req& q = s->reqs[id];
        if (q.state == REQ_REDUCING && hipEventQuery(q.done_ev) == hipSuccess) {
            complete(s, (int)id);
            acted = true;
        }
    }
    // admissions in arrival order (a request that does not fit yet does not block
    // later ones of other buckets)
    for (auto it = s->pending.begin(); it != s->pending.end();) {
        Req& q = s->reqs[*it];
        if (q.spec.arrival > t) {
            ++it;
            continue;
        }
        Pool& pl = s->pools[q.pool];
        const int c0 = find_slots(pl, q.spec.n_chains);
        const int row = c0 >= 0 ? find_row(pl) : -1;
        if (c0 < 0 || row < 0) {
            ++it;
            continue;
        }
        q.c0 = c0;
        q.row = row;
        admit(s, *it);
        it = s->pending.erase(it);
        acted = true;
    }
    // quanta: keep up to two in flight per pool with live requests
    for (int b = 0; b < (int)s->pools.size(); ++b) {
        Pool& pl = s->pools[b];
        if (pl.inflight.size() >= 2) continue;
        int hi = 0;
        bool live = false;
        for (size_t id = 0; id < s->reqs.size(); ++id) {
            const Req& q = s->reqs[id];
            if (q.pool == b && q.state == REQ_LIVE) {
                live = true;
                hi = std::max(hi, q.c0 + q.spec.n_chains);
            }
        }
        if (!live) continue;
        const int K = s->cfg.steps_per_quantum;
        run_steps(pl.p, hi, K, pl.stream);
        pl.enqueued += K;
        for (size_t id = 0; id < s->reqs.size(); ++id) {
            Req& q = s->reqs[id];
            if (q.pool == b && q.state == REQ_LIVE && q.finish_step <= pl.enqueued) enqueue_reduction(s, (int)id);
        }
        hipEvent_t e = pl.event();
        DINO_HIP(hipEventRecord(e, pl.stream));
        pl.inflight.push_back(e);
        acted = true;
    }
    return acted;
}

bool idle(const dino_server* s) {
    if (!s->pending.empty()) return false;
    for (const auto& q : s->reqs)
        if (q.state == REQ_LIVE || q.state == REQ_REDUCING) return false;
    return true;
}

}  // namespace

dino_status dino_server_create(dino_ctx* ctx, const dino_server_cfg* cfg, dino_server** out) {
    return guarded_call([&] {
        DINO_REQUIRE(ctx && cfg && out, DINO_EINVAL, "null argument");
        DINO_REQUIRE(cfg->n_buckets >= 1 && cfg->n_buckets <= DINO_MAX_BUCKETS, DINO_EINVAL,
                     "n_buckets must be in 1..DINO_MAX_BUCKETS");
        DINO_REQUIRE(cfg->max_requests >= 1, DINO_EINVAL, "max_requests must be positive");
        DINO_REQUIRE(cfg->steps_per_quantum >= 1, DINO_EINVAL, "steps_per_quantum must be positive");
        DINO_REQUIRE(cfg->dt > 0.0 && std::isfinite(cfg->dt), DINO_EINVAL, "dt must be positive");
        DINO_REQUIRE(ctx->basis.r > 0 && !ctx->layers.empty(), DINO_ESTATE,
                     "load the prior and the network before creating a server");
        for (int b = 0; b < cfg->n_buckets; ++b) {
            DINO_REQUIRE(cfg->bucket_dy[b] >= 1 && cfg->bucket_dy[b] <= ctx->d_out, DINO_EINVAL,
                         "bucket observation counts must be in 1..network outputs");
            DINO_REQUIRE(b == 0 || cfg->bucket_dy[b] > cfg->bucket_dy[b - 1], DINO_EINVAL,
                         "bucket observation counts must ascend");
            DINO_REQUIRE(cfg->bucket_slots[b] >= 1 && cfg->bucket_slots[b] <= (1 << 20), DINO_EINVAL,
                         "bucket slot counts must be in 1..2^20");
        }
        DINO_HIP(hipSetDevice(ctx->device));
        auto* s = new dino_server();
        s->ctx = ctx;
        s->cfg = *cfg;
        try {
            // admission by memory: the pools must fit the budget the caller grants
            size_t total = 0;
            for (int b = 0; b < cfg->n_buckets; ++b) {
                dino_problem_desc d{};
                d.n_chains = cfg->bucket_slots[b];
                d.d_y = cfg->bucket_dy[b];
                d.precision = cfg->precision;
                d.track_complement = cfg->track_complement;
                d.factorization = cfg->factorization;
                d.dt = cfg->dt;
                Pool pl;
                pl.dy = d.d_y;
                pl.p = create_problem(ctx, &d, cfg->max_requests, true);
                s->pools.push_back(pl);
                total += pl.p->ws_bytes;
                DINO_REQUIRE(cfg->hbm_budget_bytes <= 0.0 || (double)total <= cfg->hbm_budget_bytes, DINO_ENOMEM,
                             "the pools exceed hbm_budget_bytes: lower bucket_slots");
            }
            const int d_m = ctx->basis.d_m, r = ctx->basis.r, R = cfg->max_requests;
            for (auto& pl : s->pools) {
                DINO_HIP(hipStreamCreateWithFlags(&pl.stream, hipStreamNonBlocking));
                pl.slot_owner.assign(pl.p->C, -1);
                pl.row_owner.assign(R, -1);
                DINO_HIP(hipMalloc(&pl.d_xbar, sizeof(double) * R * r));
                DINO_HIP(hipMalloc(&pl.d_field, sizeof(double) * R * d_m));
                DINO_HIP(hipMalloc(&pl.d_counts, sizeof(int64_t) * R * 2));
                DINO_HIP(hipHostMalloc(&pl.h_rows, sizeof(double) * R * 2 * pl.dy));
                DINO_HIP(hipHostMalloc(&pl.h_field, sizeof(double) * R * d_m));
                DINO_HIP(hipHostMalloc(&pl.h_counts, sizeof(int64_t) * R * 2));
            }
        } catch (...) {
            dino_server_destroy(s);
            throw;
        }
        s->t0 = Clock::now();
        *out = s;
    });
}

dino_status dino_server_destroy(dino_server* s) {
    return guarded_call([&] {
        if (!s) return;
        (void)hipSetDevice(s->ctx->device);
        (void)hipDeviceSynchronize();
        for (auto& pl : s->pools) {
            for (auto e : pl.inflight) (void)hipEventDestroy(e);
            for (auto e : pl.spare) (void)hipEventDestroy(e);
            if (pl.stream) (void)hipStreamDestroy(pl.stream);
            if (pl.d_xbar) (void)hipFree(pl.d_xbar);
            if (pl.d_field) (void)hipFree(pl.d_field);
            if (pl.d_counts) (void)hipFree(pl.d_counts);
            if (pl.h_rows) (void)hipHostFree(pl.h_rows);
            if (pl.h_field) (void)hipHostFree(pl.h_field);
            if (pl.h_counts) (void)hipHostFree(pl.h_counts);
            destroy_problem(pl.p);
        }
        for (auto& q : s->reqs)
            if (q.done_ev) (void)hipEventDestroy(q.done_ev);
        delete s;
    });
}

dino_status dino_server_clock(const dino_server* s, double* seconds) {
    return guarded_call([&] {
        DINO_REQUIRE(s && seconds, DINO_EINVAL, "null argument");
        *seconds = s->now();
    });
}

dino_status dino_server_submit(dino_server* s, const dino_request* req) {
    return guarded_call([&] {
        DINO_REQUIRE(s && req && req->y && req->noise_var, DINO_EINVAL, "null argument");
        DINO_REQUIRE(req->d_y >= 1, DINO_EINVAL, "d_y must be positive");
        DINO_REQUIRE(req->n_steps >= 1, DINO_EINVAL, "n_steps must be positive");
        const int b = bucket_of(s, req->d_y);
        DINO_REQUIRE(b >= 0, DINO_EINVAL, "no bucket serves this many observations");
        DINO_REQUIRE(req->n_chains >= 1 && req->n_chains <= s->pools[b].p->C, DINO_EINVAL,
                     "n_chains exceeds the slots of its bucket");
        Req q;
        q.spec = *req;
        q.spec.y = nullptr;
        q.spec.noise_var = nullptr;
        q.pool = b;
        q.y.assign(req->y, req->y + req->d_y);
        q.winv.resize(req->d_y);
        for (int i = 0; i < req->d_y; ++i) {
            DINO_REQUIRE(std::isfinite(req->y[i]), DINO_ENUMERIC, "non-finite data value");
            DINO_REQUIRE(req->noise_var[i] > 0.0, DINO_EINVAL, "noise variances must be positive");
            q.winv[i] = std::isinf(req->noise_var[i]) ? 0.0 : 1.0 / std::sqrt(req->noise_var[i]);
        }
        s->reqs.push_back(std::move(q));
        s->pending.push_back((int)s->reqs.size() - 1);
    });
}

dino_status dino_server_run(dino_server* s, double until, int* n_finished) {
    return guarded_call([&] {
        DINO_REQUIRE(s, DINO_EINVAL, "null server");
        DINO_HIP(hipSetDevice(s->ctx->device));
        const size_t before = s->finished.size();
        while (!idle(s) && (until < 0.0 || s->now() < until)) {
            if (!pass(s)) std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        if (n_finished) *n_finished = (int)(s->finished.size() - before);
    });
}

dino_status dino_server_poll(dino_server* s, int max, dino_result* out, double* means, int* n) {
    return guarded_call([&] {
        DINO_REQUIRE(s && out && n && max >= 0, DINO_EINVAL, "null argument");
        const int d_m = s->ctx->basis.d_m;
        int k = 0;
        while (k < max && !s->finished.empty()) {
            Req& q = s->reqs[s->finished.front()];
            s->finished.pop_front();
            dino_result& o = out[k];
            o.request_id = q.spec.request_id;
            o.d_y = q.spec.d_y;
            o.n_chains = q.spec.n_chains;
            o.n_steps = q.spec.n_steps;
            o.arrival = q.spec.arrival;
            o.admitted = q.admitted;
            o.finished = q.finished;
            o.accepts = q.accepts;
            o.failures = q.failures;
            if (means) std::copy(q.mean.begin(), q.mean.end(), means + (size_t)k * d_m);
            q.mean.clear();
            q.mean.shrink_to_fit();
            q.state = REQ_POLLED;
            ++k;
        }
        *n = k;
    });
}

dino_status dino_server_stats(const dino_server* s, int64_t* chain_steps, int64_t* pending, int64_t* live) {
    return guarded_call([&] {
        DINO_REQUIRE(s, DINO_EINVAL, "null server");
        int64_t np = (int64_t)s->pending.size(), nl = 0;
        for (const auto& q : s->reqs)
            if (q.state == REQ_LIVE || q.state == REQ_REDUCING) ++nl;
        if (chain_steps) *chain_steps = s->chain_steps;
        if (pending) *pending = np;
        if (live) *live = nl;
    });
}
