// C ABI of the DINO-mMALA library: contexts, prior/basis, network, problems,
// the step loop, reads and stage entry points. See include/dino.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <array>
#include <exception>
#include <map>
#include <mutex>
#include <numeric>

#include "dino_internal.hpp"

namespace dino {

// Scratch of the allocation-free encode (dino_encode_noalloc): two transform buffers of
// n_fields x d_m doubles each. Host code never uses the array's name as an address: the
// device address of each GPU's copy is taken once per device by hipGetSymbolAddress
// (init_noalloc_scratch, from dino_ctx_create) and kept in g_scratch_ptr.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(16) << 20;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[MAX_DEVICES] = {};

// With `device` current: the device address of that device's scratch.
static double* init_noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    DINO_REQUIRE(device >= 0 && device < MAX_DEVICES, DINO_EINVAL, "device ordinal beyond the scratch table");
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        DINO_REQUIRE(e == hipSuccess && ptr, DINO_EDEVICE,
                     std::string("hipGetSymbolAddress of the encode scratch failed: ") + hipGetErrorString(e));
        g_scratch_ptr[device] = static_cast<double*>(ptr);
    }
    return g_scratch_ptr[device];
}

static thread_local std::string g_error;

void set_error(const std::string& msg) { g_error = msg; }
void clear_error() { g_error.clear(); }

template <typename F>
static dino_status guarded(F&& fn) {
    try {
        fn();
        return DINO_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return DINO_ENOMEM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return DINO_EDEVICE;
    } catch (...) {
        set_error("unknown failure");
        return DINO_EDEVICE;
    }
}

// Tuning table: (kind, a, b, c) -> chosen implementation and the timings it was chosen by.
struct TuneEntry {
    int choice = -1;
    std::vector<double> ms;
};
static std::mutex g_tune_mu;
static std::map<std::array<int, 4>, TuneEntry> g_tune;

int tuned_choice(int kind, int a, int b, int c) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tune.find({kind, a, b, c});
    return it == g_tune.end() ? -1 : it->second.choice;
}

void set_tuned_choice(int kind, int a, int b, int c, int choice, const std::vector<double>& ms) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    if (choice < 0) g_tune.erase({kind, a, b, c});
    else g_tune[{kind, a, b, c}] = TuneEntry{choice, ms};
}

static void free_basis(Basis& b) {
    if (b.dec) hipFree(b.dec);
    if (b.var_perp) hipFree(b.var_perp);
    if (b.lam_dev) hipFree(b.lam_dev);
    if (b.q) hipFree(b.q);
    if (b.perm) hipFree(b.perm);
    if (b.sqlam) hipFree(b.sqlam);
    if (b.UT) hipFree(b.UT);
    if (b.UT32) hipFree(b.UT32);
    if (b.lam_dis) hipFree(b.lam_dis);
    b.dec = b.var_perp = b.lam_dev = b.q = b.sqlam = b.UT = b.lam_dis = nullptr;
    b.UT32 = nullptr;
    b.perm = nullptr;
    b.dense = false;
}

static void free_layers(std::vector<Layer>& ls) {
    for (auto& l : ls) {
        if (l.W64) hipFree(l.W64);
        if (l.b64) hipFree(l.b64);
        if (l.W32) hipFree(l.W32);
        if (l.b32) hipFree(l.b32);
        if (l.WT8) hipFree(l.WT8);
    }
    ls.clear();
}

// Checks a layer chain (kinds, widths, finite values); wmax: the widest input or hidden
// width, n_act: layers with an activation.
static void validate_layers(int n_layers, const int32_t* kinds, const int32_t* fan_out, const int32_t* fan_in,
                            const double* const* W, const double* const* b, int& wmax, int& n_act) {
    DINO_REQUIRE(n_layers >= 1 && n_layers <= 16, DINO_EINVAL, "1..16 layers supported");
    DINO_REQUIRE(kinds[n_layers - 1] == DINO_LAYER_LINEAR, DINO_EINVAL, "the last layer must be linear");
    wmax = 0;
    n_act = 0;
    for (int l = 0; l < n_layers; ++l) {
        DINO_REQUIRE(kinds[l] >= 0 && kinds[l] <= 2, DINO_EINVAL, "unknown layer kind");
        DINO_REQUIRE(fan_out[l] >= 1 && fan_out[l] <= 1024 && fan_in[l] >= 1 && fan_in[l] <= 1024, DINO_EINVAL,
                     "layer widths must be in 1..1024");
        DINO_REQUIRE(W[l], DINO_EINVAL, "null weight matrix");
        if (l > 0) DINO_REQUIRE(fan_in[l] == fan_out[l - 1], DINO_EINVAL, "layer widths do not chain");
        if (kinds[l] == DINO_LAYER_RESID)
            DINO_REQUIRE(fan_in[l] == fan_out[l], DINO_EINVAL, "residual layers must be square");
        if (kinds[l] != DINO_LAYER_LINEAR) ++n_act;
        wmax = std::max(wmax, fan_in[l]);
        if (l < n_layers - 1) wmax = std::max(wmax, fan_out[l]);
        const size_t cnt = (size_t)fan_out[l] * fan_in[l];
        for (size_t e = 0; e < cnt; ++e) DINO_REQUIRE(std::isfinite(W[l][e]), DINO_ENUMERIC, "non-finite weight");
        if (b && b[l])
            for (int e = 0; e < fan_out[l]; ++e) DINO_REQUIRE(std::isfinite(b[l][e]), DINO_ENUMERIC, "non-finite bias");
    }
}

// Host copies and FP64/FP32 device copies of one layer (b may be null: zero bias).
static void upload_layer(Layer& ly, int kind, int fan_out, int fan_in, const double* W, const double* b) {
    ly.kind = kind;
    ly.fan_out = fan_out;
    ly.fan_in = fan_in;
    const size_t cnt = (size_t)ly.fan_out * ly.fan_in;
    ly.hostW.assign(W, W + cnt);
    ly.hostb.assign(ly.fan_out, 0.0);
    if (b) std::copy(b, b + ly.fan_out, ly.hostb.begin());
    std::vector<float> w32(cnt), b32(ly.fan_out);
    for (size_t e = 0; e < cnt; ++e) w32[e] = (float)ly.hostW[e];
    for (int e = 0; e < ly.fan_out; ++e) b32[e] = (float)ly.hostb[e];
    DINO_HIP(hipMalloc(&ly.W64, sizeof(double) * cnt));
    DINO_HIP(hipMalloc(&ly.b64, sizeof(double) * ly.fan_out));
    DINO_HIP(hipMalloc(&ly.W32, sizeof(float) * cnt));
    DINO_HIP(hipMalloc(&ly.b32, sizeof(float) * ly.fan_out));
    DINO_HIP(hipMemcpy(ly.W64, ly.hostW.data(), sizeof(double) * cnt, hipMemcpyHostToDevice));
    DINO_HIP(hipMemcpy(ly.b64, ly.hostb.data(), sizeof(double) * ly.fan_out, hipMemcpyHostToDevice));
    DINO_HIP(hipMemcpy(ly.W32, w32.data(), sizeof(float) * cnt, hipMemcpyHostToDevice));
    DINO_HIP(hipMemcpy(ly.b32, b32.data(), sizeof(float) * ly.fan_out, hipMemcpyHostToDevice));
}

NetView net_view(const dino_ctx* ctx) {
    NetView v{};
    v.n_layers = (int)ctx->layers.size();
    for (int l = 0; l < v.n_layers; ++l) {
        const Layer& ly = ctx->layers[l];
        v.kinds[l] = ly.kind;
        v.fan_out[l] = ly.fan_out;
        v.fan_in[l] = ly.fan_in;
        v.W64[l] = ly.W64;
        v.b64[l] = ly.b64;
        v.W32[l] = ly.W32;
        v.b32[l] = ly.b32;
    }
    return v;
}

// Carves 256-byte aligned sub-buffers out of one workspace; with base == nullptr
// it only measures.
struct Carver {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

static int ldz_of(int d_perp) { return (d_perp + 63) / 64 * 64; }

static void layout(dino_problem* p, Carver& cv) {
    const size_t C = p->C, r = p->r, dy = p->d_y, w = p->wmax;
    p->y = cv.take<double>((size_t)p->n_rows * dy);
    p->winv = cv.take<double>((size_t)p->n_rows * dy);
    p->meta.key0 = cv.take<uint64_t>(C);
    p->meta.key1 = cv.take<uint64_t>(C);
    p->meta.step = cv.take<int64_t>(C);
    p->meta.budget = cv.take<int64_t>(C);
    p->meta.burn = cv.take<int64_t>(C);
    p->meta.index = cv.take<int32_t>(C);
    p->meta.row = cv.take<int32_t>(C);
    p->meta.state = cv.take<int32_t>(C);
    p->sumx = p->serving ? cv.take<double>(C * r) : nullptr;
    p->x = cv.take<double>(C * r);
    p->g = cv.take<double>(C * r);
    p->phi = cv.take<double>(C);
    p->logdet = cv.take<double>(C);
    p->Lbuf = cv.take<double>(2 * C * (size_t)p->kdim * p->kdim);
    p->cur = cv.take<int32_t>(C);
    p->z = p->desc.track_complement ? cv.take<float>(C * (size_t)ldz_of(p->d_perp)) : nullptr;
    p->accepts = cv.take<int64_t>(C);
    p->failures = cv.take<int64_t>(C);
    p->xp = cv.take<double>(C * r);
    p->gp = cv.take<double>(C * r);
    p->phip = cv.take<double>(C);
    p->logdetp = cv.take<double>(C);
    p->okp = cv.take<int32_t>(C);
    p->lfwd = cv.take<double>(C);
    p->acc = cv.take<int32_t>(C);
    if (p->desc.method == DINO_METHOD_LAPCN) {
        p->xmap = cv.take<double>(r);
        p->Lfix = cv.take<double>(r * r);
    }
    p->f = cv.take<double>(C * dy);
    if (p->desc.precision == DINO_PREC_F64) {
        p->h0 = cv.take<double>(C * w);
        p->h1 = cv.take<double>(C * w);
        p->dprime = cv.take<double>((size_t)std::max(p->n_act, 1) * C * w);
        p->lam0 = cv.take<double>(C * dy * w);
        p->lam1 = cv.take<double>(C * dy * w);
        p->Bj = cv.take<double>(C * dy * r);
    } else {
        // the BF16 sweep reads gelu' rows of its full instance width, the FP8 sweep of the layer's
        const bool fp8 = p->desc.precision == DINO_PREC_FP8 || p->desc.precision == DINO_PREC_FP8_SINGLE;
        p->ldd32 = fp8 ? (w + 31) / 32 * 32 : 32 * sweep_nmb(p->ctx);
        p->xpf = cv.take<float>(C * r);
        p->h0f = cv.take<float>(C * w);
        p->fsync = cv.take<uint32_t>((C + 31) / 32 * 17);
        p->h1f = cv.take<float>(C * w);
        p->f32 = cv.take<float>(C * dy);
        p->d32 = cv.take<float>((size_t)std::max(p->n_act, 1) * C * p->ldd32);
        p->B16 = cv.take<__hip_bfloat16>(C * dy * ((r + 31) / 32 * 32));  // rows padded to 32
        if (p->dual) p->Bs16 = cv.take<__hip_bfloat16>(C * dy * ((r + 31) / 32 * 32));
    }
    if (p->dual && p->desc.precision == DINO_PREC_F64) p->Bs64 = cv.take<double>(C * dy * r);
    if (p->da) {
        const size_t rT = p->rT, wT = p->ctx->true_max_width;
        p->phit = cv.take<double>(C);
        p->passes = cv.take<int64_t>(C);
        p->pos = cv.take<int32_t>(C);
        p->npass = cv.take<int32_t>(1);
        p->zin = cv.take<double>(C * rT);
        if (p->ctx->basis.dense) {
            p->rowchain = cv.take<int32_t>(C);
            if (p->desc.precision == DINO_PREC_F64) {
                p->wb64 = cv.take<double>(C * (size_t)p->d_m);
                p->tp64 = cv.take<double>(C * r);
            } else {
                p->wb32 = cv.take<float>(C * (size_t)ldz_of(p->d_perp));
                p->tp32 = cv.take<float>(C * r);
            }
        }
        if (p->desc.precision == DINO_PREC_F64) {
            p->th0 = cv.take<double>(C * wT);
            p->th1 = cv.take<double>(C * wT);
            p->fT64 = cv.take<double>(C * dy);
        } else {
            p->th0f = cv.take<float>(C * wT);
            p->th1f = cv.take<float>(C * wT);
            p->fT32 = cv.take<float>(C * dy);
        }
    }
    const size_t cap = (size_t)std::max(p->desc.trace_capacity, 0);
    p->xtrace = cap ? cv.take<float>(cap * C * r) : nullptr;
    p->phitrace = cap ? cv.take<double>(cap * C) : nullptr;
}

static void check_desc(const dino_ctx* ctx, const dino_problem_desc* d) {
    DINO_REQUIRE(ctx && d, DINO_EINVAL, "null context or descriptor");
    DINO_REQUIRE(ctx->basis.r > 0, DINO_ESTATE, "load the prior before creating a problem");
    DINO_REQUIRE(!ctx->layers.empty(), DINO_ESTATE, "load the network before creating a problem");
    DINO_REQUIRE(ctx->r_in == ctx->basis.r, DINO_EINVAL, "network input width differs from the reduced dimension");
    DINO_REQUIRE(d->n_chains >= 1 && d->n_chains <= (1 << 20), DINO_EINVAL, "n_chains out of range");
    DINO_REQUIRE(d->d_y >= 1 && d->d_y <= ctx->d_out && d->d_y <= 1024, DINO_EINVAL, "d_y out of range");
    DINO_REQUIRE(d->dt > 0.0 && std::isfinite(d->dt), DINO_EINVAL, "dt must be positive");
    const bool fp8 = d->precision == DINO_PREC_FP8 || d->precision == DINO_PREC_FP8_SINGLE;
    DINO_REQUIRE(d->precision == DINO_PREC_F64 || d->precision == DINO_PREC_BF16 || fp8, DINO_EINVAL,
                 "unknown precision");
    DINO_REQUIRE(d->trace_capacity >= 0, DINO_EINVAL, "negative trace capacity");
    DINO_REQUIRE(ctx->basis.r <= 512, DINO_EINVAL, "reduced dimension above 512");
    DINO_REQUIRE(d->factorization >= DINO_FACTOR_PRIMAL && d->factorization <= DINO_FACTOR_AUTO, DINO_EINVAL,
                 "unknown factorization");
    DINO_REQUIRE(d->method >= DINO_METHOD_MMALA && d->method <= DINO_METHOD_DIS_MMALA, DINO_EINVAL, "unknown method");
    DINO_REQUIRE(d->method != DINO_METHOD_DIS_MMALA || (ctx->basis.dense && ctx->basis.lam_dis), DINO_EINVAL,
                 "DIS-mMALA needs a dense basis loaded with its DIS eigenvalues");
    if (d->method == DINO_METHOD_DA_MMALA) {
        DINO_REQUIRE(!ctx->true_layers.empty(), DINO_ESTATE, "load the true model before creating a delayed-acceptance problem");
        DINO_REQUIRE(ctx->true_r_in >= ctx->basis.r && ctx->true_r_in <= ctx->basis.d_m, DINO_EINVAL,
                     "the true model must read between r and d_m whitened coordinates");
        DINO_REQUIRE(d->d_y <= ctx->true_d_out, DINO_EINVAL, "d_y exceeds the true model's outputs");
        DINO_REQUIRE((ctx->true_r_in == ctx->basis.r && !ctx->basis.dense) || d->track_complement, DINO_EINVAL,
                     "a true model that reads complement coordinates needs track_complement");
    }
    const bool dual = d->factorization == DINO_FACTOR_DUAL ||
                      (d->factorization == DINO_FACTOR_AUTO && d->d_y < ctx->basis.r);
    DINO_REQUIRE(!dual || d->d_y <= 512, DINO_EINVAL, "the dual form factorises d_y x d_y: d_y above 512");
    DINO_REQUIRE(!dual || dual_lds_fits(ctx->basis.r, d->d_y, d->precision != DINO_PREC_F64), DINO_EINVAL,
                 "d_y x r too large for the dual form's per-chain LDS (B and the work vectors)");
    DINO_REQUIRE(d->precision != DINO_PREC_BF16 || sweep_width_ok(ctx), DINO_EINVAL,
                 "the BF16 reverse sweep holds layers of at most 512 units: this network needs the FP64 path");
    DINO_REQUIRE(!fp8 || fp8_sweep_ok(ctx, d->d_y), DINO_EINVAL,
                 "the FP8 reverse sweep holds layers of at most 800 units (and, at that width, d_y >= 5): this "
                 "network needs the FP64 path");
}

static void fill_dims(dino_problem* p, dino_ctx* ctx, const dino_problem_desc* d) {
    p->ctx = ctx;
    p->desc = *d;
    p->C = d->n_chains;
    p->r = ctx->basis.r;
    p->d_y = d->d_y;
    p->d_m = ctx->basis.d_m;
    p->d_perp = ctx->basis.dense ? p->d_m : p->d_m - p->r;  // dense: the unprojected complement draw
    p->wmax = ctx->max_width;
    p->n_act = ctx->n_act;
    p->dual = d->factorization == DINO_FACTOR_DUAL || (d->factorization == DINO_FACTOR_AUTO && d->d_y < p->r);
    p->kdim = p->dual ? p->d_y : p->r;
    p->da = d->method == DINO_METHOD_DA_MMALA;
    p->rT = p->da ? ctx->true_r_in : 0;
    p->s = (4.0 - d->dt) / (4.0 + d->dt);
    p->beta = std::sqrt(1.0 - p->s * p->s);
}

static hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Geometry stages at reduced points x (Sec. 5.1): each function is one profiled stage.
// A (slot-selected) receives I + H, later factorised in place.
static void stage_forward(dino_problem* p, int n, const double* x, double* f64, hipStream_t st) {
    if (p->desc.precision == DINO_PREC_F64) {
        launch_forward(p, n, x, f64, st);
    } else {
        launch_forward32(p, n, nullptr, x, p->f32, st);  // the first layer rounds x to FP32 as it loads
    }
}

static void stage_jacobian(dino_problem* p, int n, hipStream_t st) {
    if (p->desc.precision == DINO_PREC_F64) launch_reverse_jacobian(p, n, p->Bj, st);
    else if (p->desc.precision == DINO_PREC_FP8) launch_sweep_fp8(p, n, 2, p->d32, p->ldd32, p->B16, st);
    else if (p->desc.precision == DINO_PREC_FP8_SINGLE) launch_sweep_fp8(p, n, 1, p->d32, p->ldd32, p->B16, st);
    else launch_sweep_bf16(p, n, p->d32, p->ldd32, p->B16, st);
}

// The mixed path forms the residual and the misfit in the metric kernel (stage_hessian).
static void stage_misfit(dino_problem* p, int n, const double* f64, double* phi, double* g, hipStream_t st) {
    if (p->desc.precision == DINO_PREC_F64) launch_misfit_grad(p, n, f64, p->Bj, phi, g, st);
}

// A receives I + H (r x r), or in the dual form I + B B^T (d_y x d_y, row stride d_y).
static void stage_hessian(dino_problem* p, int n, double* phi, double* g, double* A, long strideA,
                          const int32_t* slot, int slot_xor, long slot_stride, hipStream_t st) {
    if (p->desc.precision == DINO_PREC_F64) {
        if (p->dual) launch_gram_f64(p, n, p->Bj, A, strideA, slot, slot_xor, slot_stride, st);
        else launch_gn_hessian_slot(p, n, p->Bj, A, strideA, slot, slot_xor, slot_stride, 1, 0, st);
    } else {
        if (p->dual) launch_gram_bf16(p, n, p->B16, p->f32, phi, A, strideA, slot, slot_xor, slot_stride, g, st);
        else launch_hess_bf16(p, n, p->B16, p->f32, phi, A, strideA, slot, slot_xor, slot_stride, g, st);
    }
}

// The dual form on the mixed path forms I + B B^T and factorises it in one kernel (the
// matrix stays in LDS) when the shape fits that kernel.
static bool fused_metric_factor(const dino_problem* p) {
    return p->dual && p->desc.precision != DINO_PREC_F64 && gram_chol_bf16_fits(p->r, p->d_y);
}

// I + H (or I + B B^T) into A and its factor in place, with log det and the pivot flag.
static void stage_metric_factor(dino_problem* p, int n, double* phi, double* g, double* A, long strideA,
                                const int32_t* slot, int slot_xor, long slot_stride, double* logdet, int32_t* ok,
                                hipStream_t st) {
    if (fused_metric_factor(p)) {
        launch_gram_chol_bf16(p, n, p->B16, p->f32, phi, A, strideA, slot, slot_xor, slot_stride, g, logdet, ok, 1, st);
    } else {
        stage_hessian(p, n, phi, g, A, strideA, slot, slot_xor, slot_stride, st);
        launch_cholesky_slot(n, p->kdim, A, strideA, slot, slot_xor, slot_stride, logdet, ok, st);
    }
}

static void geometry_at(dino_problem* p, int n, const double* x, double* f, double* phi, double* g, double* A,
                        long strideA, const int32_t* slot, int slot_xor, long slot_stride, double* logdet,
                        int32_t* ok, hipStream_t st) {
    stage_forward(p, n, x, f, st);
    stage_jacobian(p, n, st);
    stage_misfit(p, n, f, phi, g, st);  // the FP64 ppg reads the Jacobian
    stage_metric_factor(p, n, phi, g, A, strideA, slot, slot_xor, slot_stride, logdet, ok, st);
}

}  // namespace dino

using namespace dino;

extern "C" {

const char* dino_last_error(void) { return g_error.c_str(); }
const char* dino_version(void) { return "dino-mi355x 0.1 (gfx950)"; }

dino_status dino_ctx_create(int device, dino_ctx** out) {
    return guarded([&] {
        DINO_REQUIRE(out, DINO_EINVAL, "null output pointer");
        int count = 0;
        DINO_HIP(hipGetDeviceCount(&count));
        DINO_REQUIRE(device >= 0 && device < count, DINO_EINVAL, "device ordinal out of range");
        DINO_HIP(hipSetDevice(device));
        init_noalloc_scratch(device);
        auto* c = new dino_ctx();
        c->device = device;
        *out = c;
    });
}

dino_status dino_ctx_destroy(dino_ctx* ctx) {
    return guarded([&] {
        if (!ctx) return;
        DINO_REQUIRE(ctx->live_problems == 0, DINO_ESTATE, "context still has live problems");
        DINO_HIP(hipSetDevice(ctx->device));
        free_basis(ctx->basis);
        free_layers(ctx->layers);
        free_layers(ctx->true_layers);
        if (ctx->sweep_tiles) (void)hipFree(ctx->sweep_tiles);
        if (ctx->fp8_layers) (void)hipFree(ctx->fp8_layers);
        delete ctx;
    });
}

dino_status dino_load_prior(dino_ctx* ctx, int n, double gamma, double delta, int r) {
    return guarded([&] {
        DINO_REQUIRE(ctx, DINO_EINVAL, "null context");
        DINO_REQUIRE(ctx->live_problems == 0, DINO_ESTATE, "cannot replace the prior under live problems");
        DINO_REQUIRE(n >= 2 && n <= 1025, DINO_EINVAL, "grid size out of range");
        DINO_REQUIRE(r >= 1 && r <= n * n && r <= 512, DINO_EINVAL, "reduced dimension out of range");
        DINO_REQUIRE(gamma > 0 && delta > 0 && std::isfinite(gamma) && std::isfinite(delta), DINO_EINVAL,
                     "gamma and delta must be positive");
        DINO_HIP(hipSetDevice(ctx->device));
        // KLE order: increasing mu_k1 + mu_k2 (decreasing lambda), ties by (k1, k2).
        std::vector<double> mu(n);
        for (int k = 0; k < n; ++k) {
            const double sn = std::sin(M_PI * k / (2.0 * n));
            mu[k] = 4.0 * sn * sn;
        }
        const int d_m = n * n;
        std::vector<int> idx(d_m);
        std::iota(idx.begin(), idx.end(), 0);
        auto key = [&](int e) { int a = e / n, c = e % n; return mu[std::min(a, c)] + mu[std::max(a, c)]; };
        std::sort(idx.begin(), idx.end(), [&](int a, int b) {
            const double ka = key(a), kb = key(b);
            if (ka != kb) return ka < kb;
            return a < b;  // e = k1 * n + k2: (k1, k2) lexicographic
        });
        Basis nb;
        nb.n = n;
        nb.r = r;
        nb.d_m = d_m;
        nb.gamma = gamma;
        nb.delta = delta;
        const double h = 1.0 / (n - 1);
        for (int j = 0; j < r; ++j) {
            const int e = idx[j];
            nb.k1.push_back(e / n);
            nb.k2.push_back(e % n);
            const double a = gamma * key(e) / (h * h) + delta;
            nb.lam.push_back(1.0 / (a * a));
        }
        nb.order.assign(idx.begin(), idx.end());
        nb.sqlam_all.resize(d_m);
        for (int t = 0; t < d_m; ++t) nb.sqlam_all[t] = 1.0 / (gamma * key(idx[t]) / (h * h) + delta);
        build_basis_device(nb);
        free_basis(ctx->basis);
        ctx->basis = nb;
    });
}

dino_status dino_load_basis(dino_ctx* ctx, int r, const double* U, const double* lam_dis) {
    return guarded([&] {
        DINO_REQUIRE(ctx && U, DINO_EINVAL, "null argument");
        DINO_REQUIRE(ctx->basis.n > 0, DINO_ESTATE, "load the prior before a basis");
        DINO_REQUIRE(ctx->live_problems == 0, DINO_ESTATE, "cannot replace the basis under live problems");
        const int d_m = ctx->basis.d_m;
        DINO_REQUIRE(r >= 1 && r <= 512 && r <= d_m, DINO_EINVAL, "reduced dimension out of range");
        // orthonormal columns (the basis is H_mu-orthonormal exactly when U^T U = I)
        std::vector<double> G((size_t)r * r, 0.0);
        for (int p = 0; p < d_m; ++p) {
            const double* row = U + (size_t)p * r;
            for (int j = 0; j < r; ++j) {
                DINO_REQUIRE(std::isfinite(row[j]), DINO_ENUMERIC, "non-finite basis entry");
                for (int k = 0; k <= j; ++k) G[(size_t)j * r + k] += row[j] * row[k];
            }
        }
        for (int j = 0; j < r; ++j)
            for (int k = 0; k <= j; ++k)
                DINO_REQUIRE(std::fabs(G[(size_t)j * r + k] - (j == k ? 1.0 : 0.0)) < 1e-10, DINO_EINVAL,
                             "basis columns are not orthonormal (U^T U = I within 1e-10)");
        if (lam_dis)
            for (int j = 0; j < r; ++j)
                DINO_REQUIRE(std::isfinite(lam_dis[j]) && lam_dis[j] >= 0.0, DINO_EINVAL,
                             "DIS eigenvalues must be finite and non-negative");
        DINO_HIP(hipSetDevice(ctx->device));
        Basis& b = ctx->basis;
        // the KLE transform arrays (q, perm, sqlam, order) stay; the reduced part is replaced
        for (double** ptr : {&b.dec, &b.var_perp, &b.lam_dev, &b.UT, &b.lam_dis})
            if (*ptr) {
                (void)hipFree(*ptr);
                *ptr = nullptr;
            }
        if (b.UT32) (void)hipFree(b.UT32);
        b.UT32 = nullptr;
        b.r = r;
        b.k1.clear();
        b.k2.clear();
        b.lam.assign(lam_dis ? lam_dis : nullptr, lam_dis ? lam_dis + r : nullptr);
        build_dense_basis_device(b, std::vector<double>(U, U + (size_t)d_m * r), lam_dis);
    });
}

dino_status dino_read_basis(dino_ctx* ctx, double* dec, double* lam, double* var_perp, int32_t* modes) {
    return guarded([&] {
        DINO_REQUIRE(ctx && ctx->basis.r > 0, DINO_ESTATE, "no prior loaded");
        DINO_HIP(hipSetDevice(ctx->device));
        const Basis& b = ctx->basis;
        if (dec) DINO_HIP(hipMemcpy(dec, b.dec, sizeof(double) * (size_t)b.d_m * b.r, hipMemcpyDeviceToHost));
        if (lam) {
            if (b.dense && b.lam_dis_host.empty()) std::fill(lam, lam + b.r, 0.0);
            else std::memcpy(lam, b.dense ? b.lam_dis_host.data() : b.lam.data(), sizeof(double) * b.r);
        }
        if (var_perp) DINO_HIP(hipMemcpy(var_perp, b.var_perp, sizeof(double) * b.d_m, hipMemcpyDeviceToHost));
        if (modes)
            for (int j = 0; j < b.r; ++j) {
                modes[2 * j] = b.dense ? -1 : b.k1[j];
                modes[2 * j + 1] = b.dense ? -1 : b.k2[j];
            }
    });
}

dino_status dino_encode(dino_ctx* ctx, int n_fields, const double* fields, double* x, double* z_perp,
                        void* stream) {
    return guarded([&] {
        DINO_REQUIRE(ctx && ctx->basis.r > 0, DINO_ESTATE, "no prior loaded");
        DINO_REQUIRE(n_fields >= 1 && n_fields <= 65535 && fields && (x || z_perp), DINO_EINVAL, "bad arguments");
        DINO_HIP(hipSetDevice(ctx->device));
        const size_t nn = (size_t)ctx->basis.d_m * n_fields;
        double *t1 = nullptr, *t2 = nullptr;
        DINO_REQUIRE(hipMalloc(&t1, sizeof(double) * nn) == hipSuccess, DINO_ENOMEM, "scratch allocation failed");
        if (hipMalloc(&t2, sizeof(double) * nn) != hipSuccess) {
            (void)hipFree(t1);
            throw Error{DINO_ENOMEM, "scratch allocation failed"};
        }
        hipStream_t st = as_stream(stream);
        launch_encode(ctx->basis, n_fields, fields, x, z_perp, t1, t2, st);
        const hipError_t e = hipStreamSynchronize(st);
        (void)hipFree(t1);
        (void)hipFree(t2);
        DINO_HIP(e);
    });
}

dino_status dino_encode_noalloc(dino_ctx* ctx, int n_fields, const double* fields, double* x, double* z_perp,
                                void* stream) {
    return guarded([&] {
        DINO_REQUIRE(ctx && ctx->basis.r > 0, DINO_ESTATE, "no prior loaded");
        DINO_REQUIRE(n_fields >= 1 && n_fields <= 65535 && fields && (x || z_perp), DINO_EINVAL, "bad arguments");
        const size_t nn = (size_t)ctx->basis.d_m * n_fields;
        DINO_REQUIRE(2 * nn * sizeof(double) <= NOALLOC_SCRATCH_BYTES, DINO_EINVAL,
                     "n_fields x d_m too large for the encode scratch (2 n_fields d_m doubles must fit in " +
                         std::to_string(NOALLOC_SCRATCH_BYTES >> 20) + " MiB)");
        DINO_HIP(hipSetDevice(ctx->device));
        double* t1 = g_scratch_ptr[ctx->device];  // set by dino_ctx_create on this device
        DINO_REQUIRE(t1, DINO_ESTATE, "encode scratch not initialised on this device");
        launch_encode(ctx->basis, n_fields, fields, x, z_perp, t1, t1 + nn, as_stream(stream));
    });
}

dino_status dino_decode(dino_ctx* ctx, int n_fields, const double* x, const double* z_perp, double* fields,
                        void* stream) {
    return guarded([&] {
        DINO_REQUIRE(ctx && ctx->basis.r > 0, DINO_ESTATE, "no prior loaded");
        DINO_REQUIRE(n_fields >= 1 && n_fields <= 65535 && fields && x, DINO_EINVAL, "bad arguments");
        DINO_HIP(hipSetDevice(ctx->device));
        const size_t nn = (size_t)ctx->basis.d_m * n_fields;
        double *t1 = nullptr, *t2 = nullptr;
        DINO_REQUIRE(hipMalloc(&t1, sizeof(double) * nn) == hipSuccess, DINO_ENOMEM, "scratch allocation failed");
        if (hipMalloc(&t2, sizeof(double) * nn) != hipSuccess) {
            (void)hipFree(t1);
            throw Error{DINO_ENOMEM, "scratch allocation failed"};
        }
        hipStream_t st = as_stream(stream);
        launch_decode(ctx->basis, n_fields, x, z_perp, fields, t1, t2, st);
        const hipError_t e = hipStreamSynchronize(st);
        (void)hipFree(t1);
        (void)hipFree(t2);
        DINO_HIP(e);
    });
}

dino_status dino_load_network(dino_ctx* ctx, int n_layers, const int32_t* kinds, const int32_t* fan_out,
                              const int32_t* fan_in, const double* const* W, const double* const* b) {
    return guarded([&] {
        DINO_REQUIRE(ctx && kinds && fan_out && fan_in && W, DINO_EINVAL, "null argument");
        DINO_REQUIRE(ctx->live_problems == 0, DINO_ESTATE, "cannot replace the network under live problems");
        int wmax = 0, n_act = 0;
        validate_layers(n_layers, kinds, fan_out, fan_in, W, b, wmax, n_act);
        DINO_HIP(hipSetDevice(ctx->device));
        std::vector<Layer> ls(n_layers);
        __hip_bfloat16* new_tiles = nullptr;
        size_t n_tile_u16 = 0;
        int sweep_nmb_t = 0;
        try {
            for (int l = 0; l < n_layers; ++l) upload_layer(ls[l], kinds[l], fan_out[l], fan_in[l], W[l], b ? b[l] : nullptr);
            for (int l = 0; l + 1 < n_layers; ++l) pack_fp8_layer(ls[l]);  // the output layer stays FP32
            // BF16 MFMA operand tiles of W^T for the reverse sweep, packed for the sweep
            // instance that covers the widest layer
            dino_ctx probe;
            probe.r_in = fan_in[0];
            for (int l = 0; l < n_layers; ++l) {
                probe.layers.emplace_back();
                probe.layers.back().fan_in = fan_in[l];
                probe.layers.back().fan_out = fan_out[l];
            }
            const int nmb_t = sweep_nmb(&probe);
            sweep_nmb_t = nmb_t;
            probe.layers.clear();
            // reverse processing order: layer n_layers-2 first, output blocks ascending
            std::vector<uint16_t> all;
            for (int l = n_layers - 2; l >= 0; --l) {
                std::vector<uint16_t> tiles;
                int nmb_out = 0;
                pack_sweep_tiles(ls[l].hostW, ls[l].fan_out, ls[l].fan_in, nmb_t, tiles, nmb_out);
                all.insert(all.end(), tiles.begin(), tiles.end());
            }
            if (!all.empty()) {
                // followed by one row of 32 * nmb_t FP32 ones (the d row of layers without an
                // activation) and the output layer's rows in the sweep's register order
                n_tile_u16 = all.size();
                auto push_f32 = [&](float v) {
                    uint32_t u;
                    std::memcpy(&u, &v, 4);
                    all.push_back((uint16_t)(u & 0xFFFFu));
                    all.push_back((uint16_t)(u >> 16));
                };
                for (int e = 0; e < 32 * nmb_t; ++e) push_f32(1.f);
                std::vector<float> wpk;
                pack_sweep_wout(ls[n_layers - 1].hostW, ls[n_layers - 1].fan_out, ls[n_layers - 1].fan_in, nmb_t, wpk);
                for (float v : wpk) push_f32(v);
                DINO_HIP(hipMalloc(&new_tiles, sizeof(uint16_t) * all.size()));
                DINO_HIP(hipMemcpy(new_tiles, all.data(), sizeof(uint16_t) * all.size(), hipMemcpyHostToDevice));
            }
        } catch (...) {
            free_layers(ls);
            if (new_tiles) (void)hipFree(new_tiles);
            throw;
        }
        free_layers(ctx->layers);
        if (ctx->sweep_tiles) (void)hipFree(ctx->sweep_tiles);
        ctx->sweep_tiles = new_tiles;
        ctx->sweep_ones = new_tiles ? reinterpret_cast<const float*>(new_tiles + n_tile_u16) : nullptr;
        ctx->sweep_wout = new_tiles ? ctx->sweep_ones + 32 * sweep_nmb_t : nullptr;
        ctx->layers = std::move(ls);
        ctx->r_in = fan_in[0];
        ctx->d_out = fan_out[n_layers - 1];
        ctx->max_width = wmax;
        ctx->n_act = n_act;
        build_fp8_table(ctx);
    });
}

dino_status dino_load_true_model(dino_ctx* ctx, int n_layers, const int32_t* kinds, const int32_t* fan_out,
                                 const int32_t* fan_in, const double* const* W, const double* const* b) {
    return guarded([&] {
        DINO_REQUIRE(ctx && kinds && fan_out && fan_in && W, DINO_EINVAL, "null argument");
        DINO_REQUIRE(ctx->live_problems == 0, DINO_ESTATE, "cannot replace the true model under live problems");
        int wmax = 0, n_act = 0;
        validate_layers(n_layers, kinds, fan_out, fan_in, W, b, wmax, n_act);
        DINO_HIP(hipSetDevice(ctx->device));
        std::vector<Layer> ls(n_layers);
        try {
            for (int l = 0; l < n_layers; ++l) upload_layer(ls[l], kinds[l], fan_out[l], fan_in[l], W[l], b ? b[l] : nullptr);
        } catch (...) {
            free_layers(ls);
            throw;
        }
        free_layers(ctx->true_layers);
        ctx->true_layers = std::move(ls);
        ctx->true_r_in = fan_in[0];
        ctx->true_d_out = fan_out[n_layers - 1];
        ctx->true_max_width = wmax;
    });
}

// Every chain of a plain problem: key (seed, request id), its slot as chain index, request
// row 0, no step budget, live.
static void reset_meta(dino_problem* p, hipStream_t st) {
    launch_meta_fill(p, 0, p->C, p->desc.seed, p->desc.request_id, INT64_MAX, 0, 0, CHAIN_LIVE, 0, st);
}

extern "C++" {
namespace dino {

dino_problem* create_problem(dino_ctx* ctx, const dino_problem_desc* desc, int n_rows, bool serving) {
    check_desc(ctx, desc);
    DINO_REQUIRE(n_rows >= 1, DINO_EINVAL, "a problem needs at least one request row");
    DINO_HIP(hipSetDevice(ctx->device));
    auto* p = new dino_problem();
    try {
        fill_dims(p, ctx, desc);
        p->n_rows = n_rows;
        p->serving = serving;
        Carver cv{nullptr};
        layout(p, cv);
        const size_t need = cv.off + 256;
        hipError_t e = hipMalloc(&p->ws, need);
        DINO_REQUIRE(e == hipSuccess, DINO_ENOMEM, "device allocation of a pool workspace failed");
        p->own_ws = true;
        p->ws_bytes = need;
        Carver cv2{reinterpret_cast<char*>(p->ws)};
        layout(p, cv2);
        // every slot starts idle with zero state (the forward's counters too); rows are
        // written at admission
        DINO_HIP(hipMemset(p->ws, 0, need));
        if (p->fsync) p->fwd_chain_cap = fwd_chain_capacity(ctx->device);
        p->dinv = fused_metric_factor(p);
        launch_meta_fill(p, 0, p->C, 0, 0, 0, 0, 0, CHAIN_IDLE, 0, nullptr);
        DINO_HIP(hipDeviceSynchronize());
        p->initialised = true;
    } catch (...) {
        if (p->ws) (void)hipFree(p->ws);
        delete p;
        throw;
    }
    ctx->live_problems += 1;
    return p;
}

void destroy_problem(dino_problem* p) {
    if (!p) return;
    (void)hipSetDevice(p->ctx->device);
    (void)hipDeviceSynchronize();
    release_graphs(p);
    if (p->own_ws && p->ws) (void)hipFree(p->ws);
    for (auto& e : p->ev)
        if (e) (void)hipEventDestroy(e);
    p->ctx->live_problems -= 1;
    delete p;
}

}  // namespace dino
}  // extern "C++"

dino_status dino_problem_workspace_bytes(const dino_ctx* ctx, const dino_problem_desc* desc, size_t* bytes) {
    return guarded([&] {
        DINO_REQUIRE(bytes, DINO_EINVAL, "null output pointer");
        check_desc(ctx, desc);
        dino_problem tmp;
        fill_dims(&tmp, const_cast<dino_ctx*>(ctx), desc);
        Carver cv{nullptr};
        layout(&tmp, cv);
        *bytes = cv.off + 256;
    });
}

dino_status dino_problem_create(dino_ctx* ctx, const dino_problem_desc* desc, const double* y,
                                const double* noise_var, void* dev_ws, size_t ws_bytes, dino_problem** out) {
    return guarded([&] {
        DINO_REQUIRE(out && y && noise_var, DINO_EINVAL, "null argument");
        check_desc(ctx, desc);
        for (int i = 0; i < desc->d_y; ++i) {
            DINO_REQUIRE(std::isfinite(y[i]), DINO_ENUMERIC, "non-finite data value");
            DINO_REQUIRE(noise_var[i] > 0.0, DINO_EINVAL, "noise variances must be positive");
        }
        DINO_HIP(hipSetDevice(ctx->device));
        auto* p = new dino_problem();
        try {
            fill_dims(p, ctx, desc);
            Carver cv{nullptr};
            layout(p, cv);
            const size_t need = cv.off + 256;
            if (dev_ws) {
                DINO_REQUIRE(ws_bytes >= need, DINO_ENOMEM, "workspace smaller than dino_problem_workspace_bytes");
                DINO_REQUIRE(((uintptr_t)dev_ws & 255) == 0, DINO_EINVAL, "workspace must be 256-byte aligned");
                p->ws = dev_ws;
                p->own_ws = false;
            } else {
                hipError_t e = hipMalloc(&p->ws, need);
                DINO_REQUIRE(e == hipSuccess, DINO_ENOMEM, "device allocation of the problem workspace failed");
                p->own_ws = true;
            }
            p->ws_bytes = need;
            Carver cv2{reinterpret_cast<char*>(p->ws)};
            layout(p, cv2);
            std::vector<double> winv(desc->d_y);
            for (int i = 0; i < desc->d_y; ++i) winv[i] = std::isinf(noise_var[i]) ? 0.0 : 1.0 / std::sqrt(noise_var[i]);
            DINO_HIP(hipMemcpy(p->y, y, sizeof(double) * desc->d_y, hipMemcpyHostToDevice));
            DINO_HIP(hipMemcpy(p->winv, winv.data(), sizeof(double) * desc->d_y, hipMemcpyHostToDevice));
            if (p->d32)  // the sweep reads gelu' rows up to a multiple of 32: the padding stays zero
                DINO_HIP(hipMemset(p->d32, 0, sizeof(float) * std::max(p->n_act, 1) * p->C * p->ldd32));
            if (p->fsync) {
                DINO_HIP(hipMemset(p->fsync, 0, sizeof(uint32_t) * ((p->C + 31) / 32) * 17));
                p->fwd_chain_cap = fwd_chain_capacity(ctx->device);
            }
            p->dinv = fused_metric_factor(p);  // every factor of Lbuf then comes from the fused kernel
            reset_meta(p, nullptr);
            DINO_HIP(hipDeviceSynchronize());
        } catch (...) {
            if (p->own_ws && p->ws) hipFree(p->ws);
            delete p;
            throw;
        }
        ctx->live_problems += 1;
        *out = p;
    });
}

dino_status dino_problem_destroy(dino_problem* p) {
    return guarded([&] {
        if (!p) return;
        DINO_HIP(hipSetDevice(p->ctx->device));
        if (p->last_stream) hipStreamSynchronize(p->last_stream);
        else hipDeviceSynchronize();
        release_graphs(p);
        if (p->own_ws && p->ws) (void)hipFree(p->ws);
        for (auto& e : p->ev)
            if (e) (void)hipEventDestroy(e);
        p->ctx->live_problems -= 1;
        delete p;
    });
}

dino_status dino_chains_init(dino_problem* p, const double* x0, const float* z0, void* stream) {
    return guarded([&] {
        DINO_REQUIRE(p, DINO_EINVAL, "null problem");
        DINO_HIP(hipSetDevice(p->ctx->device));
        hipStream_t st = as_stream(stream);
        const size_t C = p->C, r = p->r;
        if (x0) {
            for (size_t e = 0; e < C * r; ++e) DINO_REQUIRE(std::isfinite(x0[e]), DINO_ENUMERIC, "non-finite x0");
            DINO_HIP(hipMemcpyAsync(p->x, x0, sizeof(double) * C * r, hipMemcpyHostToDevice, st));
        }
        if (p->z && z0) {
            const int ldz = ldz_of(p->d_perp);
            DINO_HIP(hipMemcpy2DAsync(p->z, sizeof(float) * ldz, z0, sizeof(float) * p->d_perp,
                                      sizeof(float) * p->d_perp, C, hipMemcpyHostToDevice, st));
        }
        launch_init_draws(p, x0 == nullptr, z0 == nullptr, st);
        reset_meta(p, st);
        DINO_HIP(hipMemsetAsync(p->cur, 0, sizeof(int32_t) * C, st));
        DINO_HIP(hipMemsetAsync(p->accepts, 0, sizeof(int64_t) * C, st));
        DINO_HIP(hipMemsetAsync(p->failures, 0, sizeof(int64_t) * C, st));
        const long kk = (long)p->kdim * p->kdim;
        geometry_at(p, p->C, p->x, p->f, p->phi, p->g, p->Lbuf, kk, nullptr, 0, 0, p->logdet, p->okp, st);
        if (p->dual) launch_keep_jacobian(p, p->C, st);
        if (p->da) {
            // the true misfit of the initial states (Alg. 1: known at m_j)
            DINO_HIP(hipMemsetAsync(p->passes, 0, sizeof(int64_t) * C, st));
            launch_da_init(p, p->C, st);
        }
        DINO_HIP(hipStreamSynchronize(st));
        p->step = 0;
        p->recorded = 0;
        p->initialised = true;
        p->last_stream = st;
    });
}

// Adds the stage times of the recorded ring entries to the totals (waits for the last one).
static void drain_profile(dino_problem* p) {
    if (p->ring_used == 0) return;
    const int E = DINO_N_STAGES + 1;
    DINO_HIP(hipEventSynchronize(p->ev[(p->ring_used - 1) * E + DINO_N_STAGES]));
    for (int k = 0; k < p->ring_used; ++k) {
        for (int i = 0; i < DINO_N_STAGES; ++i) {
            float ms = 0.f;
            DINO_HIP(hipEventElapsedTime(&ms, p->ev[k * E + i], p->ev[k * E + i + 1]));
            p->stage_ms[i] += ms;
        }
    }
    p->profiled_steps += p->ring_used;
    p->ring_used = 0;
}

extern "C++" {
namespace dino {

// n_steps transitions of chains [0, n) on stream st, one launch per kernel (the step
// loop that launch graphs capture).
static void run_steps_eager(dino_problem* p, int n, int n_steps, hipStream_t st) {
    const long rr = (long)p->kdim * p->kdim;
    const long half = (long)p->C * rr;
    const int L = (int)p->ctx->layers.size();
    const bool f64 = p->desc.precision == DINO_PREC_F64;
    const bool pcn = p->desc.method == DINO_METHOD_PCN || p->desc.method == DINO_METHOD_LAPCN;
    const bool lapcn = p->desc.method == DINO_METHOD_LAPCN;
    // second stage of delayed acceptance: gather, the true model's layers, decision
    const int LT = p->da ? (int)p->ctx->true_layers.size() + 2 : 0;
    const bool fused = fused_metric_factor(p);
    const int32_t launches[DINO_N_STAGES] = {1, L, f64 ? L : 1, f64 ? 1 : 0, 1, fused ? 0 : 1, 1, LT, p->z ? 1 : 0, 0};
    const bool mala = p->desc.method == DINO_METHOD_MALA || p->desc.method == DINO_METHOD_DIS_MMALA;
    const int32_t launches_pcn[DINO_N_STAGES] = {1, L, 0, 0, 0, 0, 1, 0, p->z ? 1 : 0, 0};
    // MALA: on the mixed path the misfit and ppg come from the metric kernel, told to skip the metric
    const int32_t launches_mala[DINO_N_STAGES] = {1, L, f64 ? L : 1, f64 ? 1 : 0, f64 ? 0 : 1, 0, 1, 0, p->z ? 1 : 0, 0};
    auto mark = [&](int i) {
        if (p->profile) DINO_HIP(hipEventRecord(p->ev[p->ring_used * (DINO_N_STAGES + 1) + i], st));
    };
    for (int k = 0; k < n_steps; ++k) {
        mark(0);
        if (pcn) {
            // pCN / LA-pCN baselines: proposal, network forward, misfit and decision (one kernel)
            if (lapcn) launch_lapcn_propose(p, n, st);
            else launch_pcn_propose(p, n, st);
            mark(1);
            stage_forward(p, n, p->xp, p->f, st);
            for (int i = 2; i <= 6; ++i) mark(i);
            launch_pcn_accept(p, n, st);
            mark(7);
            mark(8);
            launch_complement(p, n, st);
            mark(9);
            mark(10);
            if (p->profile) {
                for (int i = 0; i < DINO_N_STAGES; ++i) p->stage_launches[i] = launches_pcn[i];
                if (++p->ring_used == dino_problem::PROFILE_RING) drain_profile(p);
            }
            p->step += 1;
            continue;
        }
        if (mala) {
            // MALA baseline: proposal with the ppg, geometry without the factor, decision
            launch_mala_propose(p, n, st);
            mark(1);
            stage_forward(p, n, p->xp, p->f, st);
            mark(2);
            stage_jacobian(p, n, st);
            mark(3);
            stage_misfit(p, n, p->f, p->phip, p->gp, st);
            mark(4);
            if (!f64) stage_hessian(p, n, p->phip, p->gp, nullptr, 0, nullptr, 0, 0, st);  // misfit and ppg only
            mark(5);
            mark(6);
            launch_mala_accept(p, n, st);
            mark(7);
            mark(8);
            launch_complement(p, n, st);
            mark(9);
            mark(10);
            if (p->profile) {
                for (int i = 0; i < DINO_N_STAGES; ++i) p->stage_launches[i] = launches_mala[i];
                if (++p->ring_used == dino_problem::PROFILE_RING) drain_profile(p);
            }
            p->step += 1;
            continue;
        }
        if (p->dual)
            launch_propose_dual(p, n, st);
        else
            launch_propose_slot(p, n, p->x, p->g, p->Lbuf, rr, p->cur, 0, half, nullptr, true, p->xp, p->lfwd,
                                p->logdet, st);
        mark(1);
        stage_forward(p, n, p->xp, p->f, st);
        mark(2);
        stage_jacobian(p, n, st);
        mark(3);
        stage_misfit(p, n, p->f, p->phip, p->gp, st);
        mark(4);
        if (fused) {
            // one kernel for both stages (profiled as the metric stage)
            launch_gram_chol_bf16(p, n, p->B16, p->f32, p->phip, p->Lbuf, rr, p->cur, 1, half, p->gp, p->logdetp,
                                  p->okp, 1, st);
            mark(5);
        } else {
            stage_hessian(p, n, p->phip, p->gp, p->Lbuf, rr, p->cur, 1, half, st);
            mark(5);
            launch_cholesky_slot(n, p->kdim, p->Lbuf, rr, p->cur, 1, half, p->logdetp, p->okp, st);
        }
        mark(6);
        // the accept kernel also ends the step (trace row, running sums, step counter),
        // unless a second stage follows (delayed acceptance), which then ends it
        if (p->dual) launch_accept_dual(p, n, st);
        else launch_accept(p, n, st);
        mark(7);
        if (p->da) {
            launch_da_gather(p, n, st);
            launch_true_forward(p, n, p->zin, p->npass, st);
            launch_da_accept(p, n, st);
        }
        mark(8);
        launch_complement(p, n, st);
        mark(9);
        mark(10);
        if (p->profile) {
            for (int i = 0; i < DINO_N_STAGES; ++i) p->stage_launches[i] = launches[i];
            if (++p->ring_used == dino_problem::PROFILE_RING) drain_profile(p);
        }
        p->step += 1;
    }
}

void release_graphs(dino_problem* p) {
    for (auto& g : p->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    p->graphs.clear();
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    p->cap_stream = nullptr;
}

// The executable graph of `steps` transitions of chains [0, nb), captured once from the
// eager step loop on the problem's capture stream. Every kernel argument of a step is
// fixed for a problem (the trace row and the Philox counters come from the chains' own
// step counters in device memory), so one capture serves every later replay.
static hipGraphExec_t step_graph(dino_problem* p, int nb, int steps) {
    for (const auto& g : p->graphs)
        if (g.n == nb && g.steps == steps) return g.exec;
    if (!p->cap_stream) DINO_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    const int64_t step0 = p->step;
    hipGraph_t graph = nullptr;
    DINO_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed));
    try {
        run_steps_eager(p, nb, steps, p->cap_stream);
    } catch (...) {
        (void)hipStreamEndCapture(p->cap_stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        p->step = step0;
        throw;
    }
    p->step = step0;
    DINO_HIP(hipStreamEndCapture(p->cap_stream, &graph));
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    DINO_HIP(e);
    p->graphs.push_back({nb, steps, exec});
    return exec;
}

// n_steps transitions of chains [0, n) on stream st (the body of dino_step; the serving
// pools call it with n = the highest occupied slot + 1). Graph mode replays captured
// graphs of graph_steps transitions (and one of the remainder); a serving pool's chain
// count is rounded up to a bucket of 128 slots (idle slots do nothing), so a few graphs
// serve every occupancy. Profiling runs eagerly (its events sit between the stages).
void run_steps(dino_problem* p, int n, int n_steps, hipStream_t st) {
    if (n_steps > 0) {
        if (p->profile || p->launch_mode != DINO_LAUNCH_GRAPH) {
            run_steps_eager(p, n, n_steps, st);
        } else {
            const int nb = p->serving ? std::min(p->C, (n + 127) / 128 * 128) : n;
            const int G = std::max(1, std::min(p->graph_steps, n_steps));
            const hipGraphExec_t full = step_graph(p, nb, G);
            int done = 0;
            for (; done + G <= n_steps; done += G) DINO_HIP(hipGraphLaunch(full, st));
            if (done < n_steps) DINO_HIP(hipGraphLaunch(step_graph(p, nb, n_steps - done), st));
            p->step += n_steps;
        }
    }
    if (p->xtrace) p->recorded = std::min<int64_t>(p->step, p->desc.trace_capacity);
    p->last_stream = st;
}

}  // namespace dino
}  // extern "C++"

dino_status dino_set_fixed_metric(dino_problem* p, const double* x_map, const double* L_map) {
    return guarded([&] {
        DINO_REQUIRE(p && x_map && L_map, DINO_EINVAL, "null argument");
        DINO_REQUIRE(p->desc.method == DINO_METHOD_LAPCN, DINO_EINVAL, "the problem's method is not LA-pCN");
        const int r = p->r;
        for (int i = 0; i < r; ++i) {
            DINO_REQUIRE(std::isfinite(x_map[i]), DINO_ENUMERIC, "non-finite x_map");
            for (int j = 0; j <= i; ++j)
                DINO_REQUIRE(std::isfinite(L_map[(long)i * r + j]), DINO_ENUMERIC, "non-finite L_map");
            DINO_REQUIRE(L_map[(long)i * r + i] > 0.0, DINO_EINVAL, "L_map has a non-positive diagonal");
        }
        // lower triangle as given, upper triangle zero (the kernels read full rows)
        std::vector<double> L((size_t)r * r, 0.0);
        for (int i = 0; i < r; ++i)
            for (int j = 0; j <= i; ++j) L[(size_t)i * r + j] = L_map[(long)i * r + j];
        DINO_HIP(hipSetDevice(p->ctx->device));
        // steps still in flight on the problem's last stream read the fixed metric: let them
        // finish before it is overwritten (the copies below run on the null stream)
        if (p->last_stream) DINO_HIP(hipStreamSynchronize(p->last_stream));
        DINO_HIP(hipMemcpy(p->xmap, x_map, sizeof(double) * r, hipMemcpyHostToDevice));
        DINO_HIP(hipMemcpy(p->Lfix, L.data(), sizeof(double) * r * r, hipMemcpyHostToDevice));
        p->fixed_set = true;
    });
}

dino_status dino_step(dino_problem* p, int n_steps, void* stream) {
    return guarded([&] {
        DINO_REQUIRE(p, DINO_EINVAL, "null problem");
        DINO_REQUIRE(p->initialised, DINO_ESTATE, "dino_chains_init must precede dino_step");
        DINO_REQUIRE(p->desc.method != DINO_METHOD_LAPCN || p->fixed_set, DINO_ESTATE,
                     "dino_set_fixed_metric must precede dino_step for an LA-pCN problem");
        DINO_REQUIRE(n_steps >= 0, DINO_EINVAL, "negative step count");
        DINO_HIP(hipSetDevice(p->ctx->device));
        run_steps(p, p->C, n_steps, as_stream(stream));
    });
}

}  // extern "C"

// Mean milliseconds of `reps` runs of fn on st (after one untimed run).
template <typename F>
static double time_on_stream(hipStream_t st, hipEvent_t e0, hipEvent_t e1, int reps, F&& fn) {
    fn();
    DINO_HIP(hipEventRecord(e0, st));
    for (int k = 0; k < reps; ++k) fn();
    DINO_HIP(hipEventRecord(e1, st));
    DINO_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    DINO_HIP(hipEventElapsedTime(&ms, e0, e1));
    return (double)ms / reps;
}

extern "C" {

dino_status dino_autotune(dino_problem* p, void* stream, int32_t* n_entries) {
    return guarded([&] {
        DINO_REQUIRE(p && p->initialised, DINO_ESTATE, "dino_chains_init must precede dino_autotune");
        DINO_HIP(hipSetDevice(p->ctx->device));
        hipStream_t st = as_stream(stream);
        if (p->last_stream) DINO_HIP(hipStreamSynchronize(p->last_stream));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        DINO_HIP(hipEventCreate(&e0));
        DINO_HIP(hipEventCreate(&e1));
        int count = 0;
        try {
            const int C = p->C;
            const bool factor = p->desc.method == DINO_METHOD_MMALA || p->desc.method == DINO_METHOD_DA_MMALA;
            if (factor) {
                // the factor kernel at (C, k) on identity matrices in the proposal halves (scratch
                // between steps; the factor of an identity is itself, so runs can repeat)
                const int k = p->kdim;
                const long kk = (long)k * k, half = (long)C * kk;
                launch_fill_identity(C, k, p->Lbuf, kk, p->cur, 1, half, st);
                std::vector<double> ms(CHOL_VARIANTS, -1.0);
                int best = -1;
                for (int v = 0; v < CHOL_VARIANTS; ++v) {
                    if (cholesky_variant_max(v) < k) continue;
                    ms[v] = time_on_stream(st, e0, e1, 5, [&] {
                        launch_cholesky_variant(v, C, k, p->Lbuf, kk, p->cur, 1, half, p->logdetp, p->okp, st);
                    });
                    if (best < 0 || ms[v] < ms[best]) best = v;
                }
                set_tuned_choice(TUNE_CHOL, C, k, 0, best, ms);
                ++count;
            }
            const bool mixed = p->desc.precision != DINO_PREC_F64;
            if (factor && mixed && !p->dual && hess_bf16_lds_fits(p->r, p->d_y)) {
                // the Gauss-Newton kernel (LDS-staged B^T or tiles streaming B) on the Jacobian
                // at the states, into the proposal halves and proposal scratch
                stage_forward(p, C, p->x, p->f, st);
                stage_jacobian(p, C, st);
                const long kk = (long)p->r * p->r, half = (long)C * kk;
                std::vector<double> ms(2, -1.0);
                int best = -1;
                for (int cnd = 0; cnd < 2; ++cnd) {
                    set_tuned_choice(TUNE_HESS, p->r, p->d_y, 0, cnd, {});
                    ms[cnd] = time_on_stream(st, e0, e1, 5, [&] {
                        launch_hess_bf16(p, C, p->B16, p->f32, p->phip, p->Lbuf, kk, p->cur, 1, half, p->gp, st);
                    });
                    if (best < 0 || ms[cnd] < ms[best]) best = cnd;
                }
                set_tuned_choice(TUNE_HESS, p->r, p->d_y, 0, best, ms);
                ++count;
            }
            // the forward layers, one shape at a time (the other shapes at their current
            // choice), timed as the whole forward stage at the states (its outputs are scratch)
            const bool f64 = p->desc.precision == DINO_PREC_F64;
            const int kind = f64 ? TUNE_FWD64 : TUNE_FWD32;
            const int ncand = f64 ? 3 : 2;
            std::vector<std::array<int, 3>> shapes;
            const auto& L = p->ctx->layers;
            for (size_t l = 0; l < L.size(); ++l) {
                const int N = (l + 1 == L.size()) ? p->d_y : L[l].fan_out;
                const std::array<int, 3> sh{C, L[l].fan_in, N};
                if (!f64 && ((C + 31) / 32) % 8 != 0) continue;  // the block order only differs then
                if (std::find(shapes.begin(), shapes.end(), sh) == shapes.end()) shapes.push_back(sh);
            }
            // per-layer launches are timed with the one-launch forward switched off, then
            // the one launch against the best of them
            const int nl = (int)L.size();
            const bool chain = !f64 && (p->ctx->layers.size() <= 16) && p->fsync;
            if (chain) set_tuned_choice(TUNE_FWDCHAIN, C, nl, p->wmax, 0, {});
            for (const auto& sh : shapes) {
                std::vector<double> ms(ncand, -1.0);
                int best = -1;
                for (int cnd = 0; cnd < ncand; ++cnd) {
                    set_tuned_choice(kind, sh[0], sh[1], sh[2], cnd, {});
                    ms[cnd] = time_on_stream(st, e0, e1, 5, [&] { stage_forward(p, C, p->x, p->f, st); });
                    if (best < 0 || ms[cnd] < ms[best]) best = cnd;
                }
                set_tuned_choice(kind, sh[0], sh[1], sh[2], best, ms);
                ++count;
            }
            if (chain) {
                std::vector<double> ms(2, -1.0);
                ms[0] = time_on_stream(st, e0, e1, 5, [&] { stage_forward(p, C, p->x, p->f, st); });
                set_tuned_choice(TUNE_FWDCHAIN, C, nl, p->wmax, 1, {});
                if (fwd_chain_usable(p, C))
                    ms[1] = time_on_stream(st, e0, e1, 5, [&] { stage_forward(p, C, p->x, p->f, st); });
                set_tuned_choice(TUNE_FWDCHAIN, C, nl, p->wmax, (ms[1] >= 0.0 && ms[1] < ms[0]) ? 1 : 0, ms);
                ++count;
            }
        } catch (...) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        release_graphs(p);  // captured graphs hold the earlier choices
        p->last_stream = st;
        if (n_entries) *n_entries = count;
    });
}

dino_status dino_tune_set(int32_t kind, int32_t a, int32_t b, int32_t c, int32_t choice) {
    return guarded([&] {
        DINO_REQUIRE(kind >= TUNE_CHOL && kind <= TUNE_DUALSOLVE, DINO_EINVAL, "unknown tuning kind");
        const int ncand = kind == TUNE_CHOL ? CHOL_VARIANTS : (kind == TUNE_FWD64 ? 3 : 2);
        DINO_REQUIRE(choice < ncand, DINO_EINVAL, "choice out of range for this kind");
        DINO_REQUIRE(kind != TUNE_CHOL || choice < 0 || cholesky_variant_max(choice) >= b, DINO_EINVAL,
                     "factor kernel variant does not hold this order");
        DINO_REQUIRE(kind != TUNE_HESS || choice != 0 || hess_bf16_lds_fits(a, b), DINO_EINVAL,
                     "the LDS-staged Gauss-Newton kernel does not hold this shape");
        set_tuned_choice(kind, a, b, c, choice, {});
    });
}

dino_status dino_tuning_table(char* buf, size_t cap, size_t* length) {
    return guarded([&] {
        std::string out;
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            for (const auto& kv : g_tune) {
                out += std::to_string(kv.first[0]) + " " + std::to_string(kv.first[1]) + " " +
                       std::to_string(kv.first[2]) + " " + std::to_string(kv.first[3]) + " " +
                       std::to_string(kv.second.choice);
                for (double m : kv.second.ms) out += " " + std::to_string(m);
                out += "\n";
            }
        }
        if (length) *length = out.size();
        if (buf && cap) {
            const size_t n = std::min(cap - 1, out.size());
            std::memcpy(buf, out.data(), n);
            buf[n] = 0;
        }
    });
}

dino_status dino_set_launch_mode(dino_problem* p, int mode, int steps_per_graph) {
    return guarded([&] {
        DINO_REQUIRE(p, DINO_EINVAL, "null problem");
        DINO_REQUIRE(mode == DINO_LAUNCH_EAGER || mode == DINO_LAUNCH_GRAPH, DINO_EINVAL, "unknown launch mode");
        DINO_REQUIRE(steps_per_graph >= 1 && steps_per_graph <= 256, DINO_EINVAL, "steps_per_graph must be in 1..256");
        DINO_HIP(hipSetDevice(p->ctx->device));
        if (p->last_stream) DINO_HIP(hipStreamSynchronize(p->last_stream));
        if (steps_per_graph != p->graph_steps) release_graphs(p);
        p->launch_mode = mode;
        p->graph_steps = steps_per_graph;
    });
}

dino_status dino_set_profiling(dino_problem* p, int enable) {
    return guarded([&] {
        DINO_REQUIRE(p, DINO_EINVAL, "null problem");
        DINO_HIP(hipSetDevice(p->ctx->device));
        if (enable && p->ev.empty()) {
            p->ev.assign((size_t)dino_problem::PROFILE_RING * (DINO_N_STAGES + 1), nullptr);
            for (auto& e : p->ev) DINO_HIP(hipEventCreate(&e));
        }
        if (p->profile) drain_profile(p);
        p->profile = enable != 0;
        p->ring_used = 0;
        for (int i = 0; i < DINO_N_STAGES; ++i) {
            p->stage_ms[i] = 0.0;
            p->stage_launches[i] = 0;
        }
        p->profiled_steps = 0;
    });
}

dino_status dino_read_profile(dino_problem* p, double* stage_ms, int32_t* launches, int64_t* steps) {
    return guarded([&] {
        DINO_REQUIRE(p, DINO_EINVAL, "null problem");
        if (!p->ev.empty()) {
            DINO_HIP(hipSetDevice(p->ctx->device));
            drain_profile(p);
        }
        for (int i = 0; i < DINO_N_STAGES; ++i) {
            if (stage_ms) stage_ms[i] = p->stage_ms[i];
            if (launches) launches[i] = p->stage_launches[i];
        }
        if (steps) *steps = p->profiled_steps;
    });
}

const char* dino_stage_name(int stage) {
    static const char* names[DINO_N_STAGES] = {"proposal", "forward", "jacobian", "misfit_ppg", "gn_hessian",
                                               "cholesky", "accept", "second_stage", "complement", "trace"};
    return (stage >= 0 && stage < DINO_N_STAGES) ? names[stage] : "";
}

dino_status dino_read_states(dino_problem* p, double* x, float* z) {
    return guarded([&] {
        DINO_REQUIRE(p && p->initialised, DINO_ESTATE, "problem not initialised");
        DINO_HIP(hipSetDevice(p->ctx->device));
        DINO_HIP(hipStreamSynchronize(p->last_stream));
        if (x) DINO_HIP(hipMemcpy(x, p->x, sizeof(double) * p->C * p->r, hipMemcpyDeviceToHost));
        if (z) {
            DINO_REQUIRE(p->z, DINO_ESTATE, "complement not tracked");
            DINO_HIP(hipMemcpy2D(z, sizeof(float) * p->d_perp, p->z, sizeof(float) * ldz_of(p->d_perp),
                                 sizeof(float) * p->d_perp, p->C, hipMemcpyDeviceToHost));
        }
    });
}

dino_status dino_read_cache(dino_problem* p, double* phi, double* g, double* L) {
    return guarded([&] {
        DINO_REQUIRE(p && p->initialised, DINO_ESTATE, "problem not initialised");
        DINO_HIP(hipSetDevice(p->ctx->device));
        DINO_HIP(hipStreamSynchronize(p->last_stream));
        if (phi) DINO_HIP(hipMemcpy(phi, p->phi, sizeof(double) * p->C, hipMemcpyDeviceToHost));
        if (g) DINO_HIP(hipMemcpy(g, p->g, sizeof(double) * p->C * p->r, hipMemcpyDeviceToHost));
        if (L) {
            std::vector<int32_t> cur(p->C);
            DINO_HIP(hipMemcpy(cur.data(), p->cur, sizeof(int32_t) * p->C, hipMemcpyDeviceToHost));
            const size_t rr = (size_t)p->r * p->r, kk = (size_t)p->kdim * p->kdim;
            for (int c = 0; c < p->C; ++c)
                DINO_HIP(hipMemcpy(L + c * rr, p->Lbuf + ((size_t)cur[c] * p->C + c) * kk, sizeof(double) * kk,
                                   hipMemcpyDeviceToHost));
        }
    });
}

dino_status dino_read_diagnostics(dino_problem* p, int64_t* accepts, int64_t* failures, int64_t* steps) {
    return guarded([&] {
        DINO_REQUIRE(p && p->initialised, DINO_ESTATE, "problem not initialised");
        DINO_HIP(hipSetDevice(p->ctx->device));
        DINO_HIP(hipStreamSynchronize(p->last_stream));
        if (accepts) DINO_HIP(hipMemcpy(accepts, p->accepts, sizeof(int64_t) * p->C, hipMemcpyDeviceToHost));
        if (failures) DINO_HIP(hipMemcpy(failures, p->failures, sizeof(int64_t) * p->C, hipMemcpyDeviceToHost));
        if (steps) *steps = p->step;
    });
}

dino_status dino_read_delayed(dino_problem* p, double* phi_true, int64_t* passes) {
    return guarded([&] {
        DINO_REQUIRE(p && p->initialised, DINO_ESTATE, "problem not initialised");
        DINO_REQUIRE(p->da, DINO_EINVAL, "not a delayed-acceptance problem");
        DINO_HIP(hipSetDevice(p->ctx->device));
        DINO_HIP(hipStreamSynchronize(p->last_stream));
        if (phi_true) DINO_HIP(hipMemcpy(phi_true, p->phit, sizeof(double) * p->C, hipMemcpyDeviceToHost));
        if (passes) DINO_HIP(hipMemcpy(passes, p->passes, sizeof(int64_t) * p->C, hipMemcpyDeviceToHost));
    });
}

dino_status dino_eval_true_misfit(dino_problem* p, int n, const double* z_in, double* phi_true, void* stream) {
    return guarded([&] {
        DINO_REQUIRE(p && z_in && phi_true, DINO_EINVAL, "null argument");
        DINO_REQUIRE(p->da, DINO_EINVAL, "not a delayed-acceptance problem");
        DINO_REQUIRE(n >= 1 && n <= p->C, DINO_EINVAL, "n out of range");
        DINO_HIP(hipSetDevice(p->ctx->device));
        hipStream_t st = as_stream(stream);
        launch_true_forward(p, n, z_in, nullptr, st);
        launch_true_misfit(p, n, phi_true, st);
        p->last_stream = st;
    });
}

dino_status dino_read_trace(dino_problem* p, float* x_trace, double* phi_trace, int64_t* n_recorded) {
    return guarded([&] {
        DINO_REQUIRE(p && p->initialised, DINO_ESTATE, "problem not initialised");
        DINO_HIP(hipSetDevice(p->ctx->device));
        DINO_HIP(hipStreamSynchronize(p->last_stream));
        if (n_recorded) *n_recorded = p->recorded;
        if (p->recorded == 0) return;
        if (x_trace)
            DINO_HIP(hipMemcpy(x_trace, p->xtrace, sizeof(float) * p->recorded * p->C * p->r, hipMemcpyDeviceToHost));
        if (phi_trace)
            DINO_HIP(hipMemcpy(phi_trace, p->phitrace, sizeof(double) * p->recorded * p->C, hipMemcpyDeviceToHost));
    });
}

dino_status dino_posterior(dino_problem* p, int burn_in, double* mean, double* var, double* xbar, double* S) {
    return guarded([&] {
        DINO_REQUIRE(p && p->initialised, DINO_ESTATE, "problem not initialised");
        DINO_REQUIRE(burn_in >= 0 && burn_in < p->recorded, DINO_EINVAL, "burn_in must leave recorded steps");
        DINO_HIP(hipSetDevice(p->ctx->device));
        hipStream_t st = p->last_stream;
        const int r = p->r, d_m = p->d_m;
        double *dm = nullptr, *dv = nullptr, *dx = nullptr, *dS = nullptr;
        DINO_HIP(hipMalloc(&dm, sizeof(double) * d_m));
        DINO_HIP(hipMalloc(&dv, sizeof(double) * d_m));
        DINO_HIP(hipMalloc(&dx, sizeof(double) * r));
        DINO_HIP(hipMalloc(&dS, sizeof(double) * r * r));
        launch_posterior(p, burn_in, dm, dv, dx, dS, st);
        DINO_HIP(hipStreamSynchronize(st));
        if (mean) DINO_HIP(hipMemcpy(mean, dm, sizeof(double) * d_m, hipMemcpyDeviceToHost));
        if (var) DINO_HIP(hipMemcpy(var, dv, sizeof(double) * d_m, hipMemcpyDeviceToHost));
        if (xbar) DINO_HIP(hipMemcpy(xbar, dx, sizeof(double) * r, hipMemcpyDeviceToHost));
        if (S) DINO_HIP(hipMemcpy(S, dS, sizeof(double) * r * r, hipMemcpyDeviceToHost));
        hipFree(dm);
        hipFree(dv);
        hipFree(dx);
        hipFree(dS);
    });
}

dino_status dino_ess(dino_problem* p, int burn_in, double* ess) {
    return guarded([&] {
        DINO_REQUIRE(p && p->initialised && ess, DINO_EINVAL, "bad arguments");
        DINO_REQUIRE(burn_in >= 0 && p->recorded - burn_in >= 2, DINO_EINVAL, "need two recorded steps after burn_in");
        DINO_HIP(hipSetDevice(p->ctx->device));
        double* d = nullptr;
        DINO_HIP(hipMalloc(&d, sizeof(double) * p->r));
        launch_ess(p, burn_in, d, p->last_stream);
        DINO_HIP(hipMemcpy(ess, d, sizeof(double) * p->r, hipMemcpyDeviceToHost));
        hipFree(d);
    });
}

dino_status dino_eval_geometry(dino_problem* p, int n, const double* x, double* f, double* phi, double* g,
                               double* H, double* L, double* logdet, int32_t* ok, void* stream) {
    return guarded([&] {
        DINO_REQUIRE(p && x && f && phi && g && L && logdet && ok, DINO_EINVAL, "null argument");
        DINO_REQUIRE(n >= 1 && n <= p->C, DINO_EINVAL, "n out of range");
        DINO_HIP(hipSetDevice(p->ctx->device));
        hipStream_t st = as_stream(stream);
        const long rr = (long)p->r * p->r;
        stage_forward(p, n, x, f, st);
        stage_jacobian(p, n, st);
        stage_misfit(p, n, f, phi, g, st);
        if (fused_metric_factor(p)) {
            launch_gram_chol_bf16(p, n, p->B16, p->f32, phi, L, rr, nullptr, 0, 0, g, logdet, ok, 0, st);
            if (p->desc.precision != DINO_PREC_F64) launch_to_double((long)n * p->d_y, p->f32, f, st);
            if (H) launch_btb(p, n, H, st);
        } else {
            stage_hessian(p, n, phi, g, L, rr, nullptr, 0, 0, st);
            if (p->desc.precision != DINO_PREC_F64) launch_to_double((long)n * p->d_y, p->f32, f, st);
            if (H) {
                if (p->dual) launch_btb(p, n, H, st);
                else launch_sym_from_lower(n, p->r, L, H, st);
            }
            launch_cholesky_slot(n, p->kdim, L, rr, nullptr, 0, 0, logdet, ok, st);
        }
        p->last_stream = st;
    });
}

dino_status dino_eval_propose(dino_problem* p, int n, const double* x, const double* g, const double* L,
                              const double* xi, double* xp, void* stream) {
    return guarded([&] {
        DINO_REQUIRE(p && x && g && L && xi && xp, DINO_EINVAL, "null argument");
        DINO_REQUIRE(!p->dual, DINO_EINVAL, "dino_eval_propose serves the primal form");
        DINO_REQUIRE(n >= 1 && n <= p->C, DINO_EINVAL, "n out of range");
        DINO_HIP(hipSetDevice(p->ctx->device));
        hipStream_t st = as_stream(stream);
        launch_propose_slot(p, n, x, g, L, (long)p->r * p->r, nullptr, 0, 0, xi, false, xp, nullptr, nullptr, st);
        p->last_stream = st;
    });
}

dino_status dino_eval_log_rho(dino_problem* p, int n, const double* x, const double* phi_x, const double* g_x,
                              const double* L_x, const double* logdet_x, const double* xp, const double* phi_p,
                              const double* g_p, const double* L_p, const double* logdet_p, double* log_rho,
                              void* stream) {
    return guarded([&] {
        DINO_REQUIRE(p && x && phi_x && g_x && L_x && logdet_x && xp && phi_p && g_p && L_p && logdet_p && log_rho,
                     DINO_EINVAL, "null argument");
        DINO_REQUIRE(!p->dual, DINO_EINVAL, "dino_eval_log_rho serves the primal form");
        DINO_REQUIRE(n >= 1 && n <= p->C, DINO_EINVAL, "n out of range");
        DINO_HIP(hipSetDevice(p->ctx->device));
        hipStream_t st = as_stream(stream);
        launch_log_rho(p, n, x, phi_x, g_x, L_x, logdet_x, xp, phi_p, g_p, L_p, logdet_p, log_rho, st);
        p->last_stream = st;
    });
}

dino_status dino_eval_jacobian(dino_problem* p, int n, const double* x, double* B, void* stream) {
    return guarded([&] {
        DINO_REQUIRE(p && x && B, DINO_EINVAL, "null argument");
        DINO_REQUIRE(n >= 1 && n <= p->C, DINO_EINVAL, "n out of range");
        DINO_HIP(hipSetDevice(p->ctx->device));
        hipStream_t st = as_stream(stream);
        stage_forward(p, n, x, p->f, st);
        stage_jacobian(p, n, st);
        launch_jacobian_to_double(p, n, B, st);
        p->last_stream = st;
    });
}

dino_status dino_jacobian_ld(const dino_problem* p, int32_t* ldb) {
    return guarded([&] {
        DINO_REQUIRE(p && ldb, DINO_EINVAL, "null argument");
        *ldb = jacobian_ld(p);
    });
}

dino_status dino_eval_propose_dual(dino_problem* p, int n, const double* x, const double* g, const void* B,
                                   const double* K, const double* logdet, const double* xi, double* xp, double* lfwd,
                                   void* stream) {
    return guarded([&] {
        DINO_REQUIRE(p && x && g && B && K && logdet && xi && xp && lfwd, DINO_EINVAL, "null argument");
        DINO_REQUIRE(p->dual, DINO_EINVAL, "dino_eval_propose_dual serves the dual form");
        DINO_REQUIRE(p->desc.method == DINO_METHOD_MMALA, DINO_EINVAL, "dino_eval_propose_dual serves mMALA problems");
        DINO_REQUIRE(n >= 1 && n <= p->C, DINO_EINVAL, "n out of range");
        DINO_HIP(hipSetDevice(p->ctx->device));
        hipStream_t st = as_stream(stream);
        launch_eval_propose_dual(p, n, x, g, B, K, logdet, xi, xp, lfwd, st);
        p->last_stream = st;
    });
}

dino_status dino_eval_log_rho_dual(dino_problem* p, int n, const double* x, const double* phi_x, const double* g_x,
                                   const void* B_x, const double* K_x, const double* logdet_x, const double* xp,
                                   const double* phi_p, const double* g_p, const void* B_p, const double* K_p,
                                   const double* logdet_p, double* log_rho, void* stream) {
    return guarded([&] {
        DINO_REQUIRE(p && x && phi_x && g_x && B_x && K_x && logdet_x && xp && phi_p && g_p && B_p && K_p &&
                         logdet_p && log_rho,
                     DINO_EINVAL, "null argument");
        DINO_REQUIRE(p->dual, DINO_EINVAL, "dino_eval_log_rho_dual serves the dual form");
        DINO_REQUIRE(p->desc.method == DINO_METHOD_MMALA, DINO_EINVAL, "dino_eval_log_rho_dual serves mMALA problems");
        DINO_REQUIRE(n >= 1 && n <= p->C, DINO_EINVAL, "n out of range");
        DINO_HIP(hipSetDevice(p->ctx->device));
        hipStream_t st = as_stream(stream);
        launch_eval_log_rho_dual(p, n, x, phi_x, g_x, B_x, K_x, logdet_x, xp, phi_p, g_p, B_p, K_p, logdet_p, log_rho,
                                 st);
        p->last_stream = st;
    });
}

dino_status dino_eval_normals(dino_problem* p, int n, int stream_id, int64_t step, int count, double* out,
                              void* stream) {
    return guarded([&] {
        DINO_REQUIRE(p && out, DINO_EINVAL, "null argument");
        DINO_REQUIRE(n >= 1 && count >= 1 && stream_id >= 0 && step >= 0, DINO_EINVAL, "bad sizes");
        DINO_HIP(hipSetDevice(p->ctx->device));
        hipStream_t st = as_stream(stream);
        launch_normals(p->desc.seed, p->desc.request_id, n, stream_id, step, count, out, st);
        p->last_stream = st;
    });
}

}  // extern "C"
