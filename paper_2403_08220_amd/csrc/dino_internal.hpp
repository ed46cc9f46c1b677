// Internal declarations of the DINO-mMALA HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>
#include <exception>
#include <new>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dino.h"

namespace dino {

// Largest grid extent in y and z; kernels that put chains (or fields) there loop over
// c = blockIdx.y + k gridDim.y, so any count fits.
constexpr unsigned GRID_Y_MAX = 65535;
inline unsigned grid_y(long n) { return (unsigned)(n < (long)GRID_Y_MAX ? (n > 0 ? n : 1) : GRID_Y_MAX); }

// ----------------------------------------------------------------------------------
// Errors: every ABI call converts failures to a status and a thread-local message.
struct Error {
    dino_status code;
    std::string msg;
};

void set_error(const std::string& msg);
void clear_error();

#define DINO_HIP(call)                                                                         \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            throw ::dino::Error{DINO_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define DINO_REQUIRE(cond, code, text)                                \
    do {                                                              \
        if (!(cond)) throw ::dino::Error{(code), std::string(text)}; \
    } while (0)

// Runs fn and converts any failure into a status and the thread's error message.
template <typename F>
inline dino_status guarded_call(F&& fn) {
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

// ----------------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11). Counter (block, stream, step, chain),
// key (seed, request id). Both the oracle and the kernels implement it from that
// definition; streams: 0 proposal normals, 1 complement normals, 2 MH uniform,
// 3 initial x, 4 initial z.
enum : int {
    STREAM_XI = 0,
    STREAM_COMPLEMENT = 1,
    STREAM_UNIFORM = 2,
    STREAM_INIT_X = 3,
    STREAM_INIT_Z = 4,
    STREAM_UNIFORM2 = 5  // the second-stage uniform of delayed acceptance
};

constexpr uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t PHILOX_M1 = 0xCA5A826395121157ull;
constexpr uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t PHILOX_W1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        if (i) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        const uint64_t hi0 = __umul64hi(PHILOX_M0, c[0]);
        const uint64_t lo0 = PHILOX_M0 * c[0];
        const uint64_t hi1 = __umul64hi(PHILOX_M1, c[2]);
        const uint64_t lo1 = PHILOX_M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0;
        const uint64_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// ((w >> 12) + 1/2) 2^-52: exact in double, strictly inside (0, 1).
__device__ __forceinline__ double philox_u01(uint64_t w) { return ((double)(w >> 12) + 0.5) * 0x1p-52; }

// Normals 4*block .. 4*block+3 of a stream (Box-Muller on word pairs (0,1), (2,3)).
__device__ __forceinline__ void philox_normals4(uint64_t seed, uint64_t rid, uint64_t block, uint64_t stream,
                                                uint64_t step, uint64_t chain, double out[4]) {
    uint64_t c[4] = {block, stream, step, chain};
    philox4x64(c, seed, rid);
    const double u0 = philox_u01(c[0]), u1 = philox_u01(c[1]);
    const double u2 = philox_u01(c[2]), u3 = philox_u01(c[3]);
    const double R0 = sqrt(-2.0 * log(u0));
    const double R2 = sqrt(-2.0 * log(u2));
    double s1, c1, s3, c3;
    sincos(2.0 * M_PI * u1, &s1, &c1);
    sincos(2.0 * M_PI * u3, &s3, &c3);
    out[0] = R0 * c1;
    out[1] = R0 * s1;
    out[2] = R2 * c3;
    out[3] = R2 * s3;
}

__device__ __forceinline__ double philox_uniform(uint64_t seed, uint64_t rid, uint64_t step, uint64_t chain) {
    uint64_t c[4] = {0, (uint64_t)STREAM_UNIFORM, step, chain};
    philox4x64(c, seed, rid);
    return philox_u01(c[0]);
}

// Word 0 of block 0 of `stream` at (step, chain) as a uniform in (0, 1).
__device__ __forceinline__ double philox_uniform_stream(uint64_t seed, uint64_t rid, int stream, uint64_t step,
                                                        uint64_t chain) {
    uint64_t c[4] = {0, (uint64_t)stream, step, chain};
    philox4x64(c, seed, rid);
    return philox_u01(c[0]);
}

// The pCN move of one FP32 complement coordinate, z+ = s z + beta zeta, rounded to FP32;
// every kernel that forms z+ uses this one expression, so they agree bit for bit.
__device__ __forceinline__ float pcn_move(float z, double zeta, double s, double beta) {
    return (float)fma(beta, zeta, s * (double)z);
}

// ----------------------------------------------------------------------------------
// Per-chain stream keys and life cycle (device arrays, one entry per chain slot). A
// plain problem fills them uniformly (key (seed, request id), index = slot, row 0,
// every chain live); a serving pool sets them per request when it admits one.
enum : int32_t { CHAIN_IDLE = 0, CHAIN_LIVE = 1, CHAIN_FRESH = 2 };

struct ChainMeta {
    uint64_t* key0 = nullptr;  // Philox key word 0 (seed)
    uint64_t* key1 = nullptr;  // Philox key word 1 (request id)
    int64_t* step = nullptr;   // Markov steps taken: the counter's step field
    int64_t* budget = nullptr; // the chain stops (goes idle) after this many steps
    int64_t* burn = nullptr;   // steps before the running sums start
    int32_t* index = nullptr;  // chain index inside its request: the counter's chain field
    int32_t* row = nullptr;    // request row of y and Gamma^-1/2
    int32_t* state = nullptr;  // CHAIN_IDLE / CHAIN_LIVE / CHAIN_FRESH (joins at the next step)
};

__device__ __forceinline__ int32_t chain_row(const ChainMeta& m, int c) { return m.row ? m.row[c] : 0; }
__device__ __forceinline__ int32_t chain_state(const ChainMeta& m, int c) {
    return m.state ? m.state[c] : (int32_t)CHAIN_LIVE;
}

// FP64 value of a stored Jacobian entry (FP64 path or BF16 path).
__device__ __forceinline__ double to_d(double v) { return v; }
__device__ __forceinline__ double to_d(__hip_bfloat16 v) { return (double)__bfloat162float(v); }

// ----------------------------------------------------------------------------------
// Host-side objects.
struct Layer {
    int kind;
    int fan_out, fan_in;
    double* W64 = nullptr;  // fan_out x fan_in
    double* b64 = nullptr;
    float* W32 = nullptr;
    float* b32 = nullptr;
    std::vector<double> hostW, hostb;
    // FP8 e4m3 W^T for the FP8 reverse sweep (fan_in rounded up to 32 rows, fan_out to kp8 = a
    // multiple of 64, zero padded) in the sweep's operand order (32 x 64 blocks of 2 KB),
    // followed in the same allocation by the E8M0 column exponents (wexp8, one per row, 127
    // on the zero rows)
    uint8_t* WT8 = nullptr;
    uint8_t* wexp8 = nullptr;
    int kp8 = 0;
};

struct Basis {
    int n = 0, r = 0, d_m = 0;
    double gamma = 0, delta = 0;
    std::vector<int32_t> k1, k2;   // kept modes
    std::vector<double> lam;       // kept eigenvalues
    std::vector<int32_t> order;    // all d_m modes (k1 n + k2) in KLE order
    std::vector<double> sqlam_all; // sqrt(lambda) in KLE order
    double* dec = nullptr;         // d_m x r
    double* var_perp = nullptr;    // d_m
    double* lam_dev = nullptr;     // r
    double* q = nullptr;           // n x n DCT-II matrix Q[i][k] = q_k(i)
    int32_t* perm = nullptr;       // d_m: order on the device
    double* sqlam = nullptr;       // d_m: sqrt_lam_all on the device
    // dense basis (dino_load_basis): orthonormal u_j in whitened coordinates (KLE order);
    // the reduced coordinates are x = U^T z and a problem's complement state is the
    // unprojected w in R^d_m, whose complement part is (I - U U^T) w
    bool dense = false;
    double* UT = nullptr;          // r x d_m FP64, row j = u_j
    float* UT32 = nullptr;         // r x d_m FP32 copy (mixed path)
    double* lam_dis = nullptr;     // r DIS eigenvalues (device), null when none were given
    std::vector<double> lam_dis_host;
};

// One layer of the FP8 reverse sweep, in processing order (output side first).
struct Fp8SweepLayer {
    const uint8_t* WT;    // FP8 W^T in operand order (rows: fan_in rounded up to 32; K: kp)
    const uint8_t* wexp;  // E8M0 column exponents, one per row of WT
    int K, N, kp;         // fan_out, fan_in, K rounded up to 64
    int resid;            // Lambda <- Lambda + ...
    int act;              // index of the layer's gelu' rows among the activated layers, -1 if linear
    int rows;             // rows of WT: fan_in rounded up to 32
};

struct dino_ctx_impl;
}  // namespace dino

struct dino_ctx {
    int device = 0;
    dino::Basis basis;
    std::vector<dino::Layer> layers;
    int r_in = 0, d_out = 0, max_width = 0, n_act = 0;
    int live_problems = 0;
    __hip_bfloat16* sweep_tiles = nullptr;  // BF16 W^T tiles of the reverse sweep, in work-item order
    const float* sweep_ones = nullptr;      // 32 * nmb FP32 ones after the tiles (same allocation)
    const float* sweep_wout = nullptr;      // output layer rows in the sweep's register order (same allocation)
    dino::Fp8SweepLayer* fp8_layers = nullptr;  // device table of the FP8 sweep's layers
    // true-model stand-in of delayed acceptance: a network on the first r_T whitened
    // coordinates of the full parameter (FP64 and FP32 copies)
    std::vector<dino::Layer> true_layers;
    int true_r_in = 0, true_d_out = 0, true_max_width = 0;
};

namespace dino {

// Device views used by launches.
struct NetView {
    int n_layers;
    int kinds[16];
    int fan_out[16];
    int fan_in[16];
    const double* W64[16];
    const double* b64[16];
    const float* W32[16];
    const float* b32[16];
};

}  // namespace dino

struct dino_problem {
    dino_ctx* ctx = nullptr;
    dino_problem_desc desc{};
    int C = 0, r = 0, d_y = 0, d_m = 0, d_perp = 0, wmax = 0, n_act = 0;
    double s = 0, beta = 0;
    bool own_ws = false;
    bool initialised = false;
    bool serving = false;     // a serving pool: per-request rows, running sums
    bool fixed_set = false;   // LA-pCN: dino_set_fixed_metric has been called
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int64_t step = 0;
    int64_t recorded = 0;
    hipStream_t last_stream = nullptr;

    // problem data: one row per request (a plain problem has one)
    int n_rows = 1;
    double* y = nullptr;      // n_rows x d_y
    double* winv = nullptr;   // n_rows x d_y: Gamma^-1/2 diagonal (0 for unobserved outputs)
    dino::ChainMeta meta;     // per-chain keys, steps and life cycle
    double* sumx = nullptr;   // C x r running sums of x after burn-in (serving pools)
    // chain state and its cache
    double* x = nullptr;      // C x r
    double* g = nullptr;      // C x r
    double* phi = nullptr;    // C
    double* logdet = nullptr; // C
    double* Lbuf = nullptr;   // 2 x C x r x r (ping-pong)
    int32_t* cur = nullptr;   // C: which half of Lbuf holds the state's factor
    float* z = nullptr;       // C x d_perp
    int64_t* accepts = nullptr;
    int64_t* failures = nullptr;
    // proposal scratch
    double* xp = nullptr;
    double* gp = nullptr;
    double* phip = nullptr;
    double* logdetp = nullptr;
    int32_t* okp = nullptr;
    double* lfwd = nullptr;   // log rho_0(x -> xp) per chain (LA-pCN: its density term)
    double* xmap = nullptr;   // LA-pCN: r, the MAP
    double* Lfix = nullptr;   // LA-pCN: r x r, the factor of I + H(x_map)
    int32_t* acc = nullptr;   // accept flag of the last step
    double* f = nullptr;      // C x d_y (FP64)
    double* h0 = nullptr;     // C x wmax activations (ping)
    double* h1 = nullptr;     // C x wmax (pong)
    double* dprime = nullptr; // n_act x C x wmax  gelu'(z) of every activated layer
    double* lam0 = nullptr;   // C x d_y x wmax   reverse-sweep buffers (FP64 path)
    double* lam1 = nullptr;
    double* Bj = nullptr;     // C x d_y x r whitened reduced Jacobian Gamma^-1/2 J
    // mixed-precision path buffers
    int ldd32 = 0;            // row length of d32 (width rounded up to 32)
    float* xpf = nullptr;     // C x r reduced point in FP32
    float* h0f = nullptr;     // C x wmax FP32 activations
    uint32_t* fsync = nullptr;  // row-block counters of the one-launch FP32 forward (zero between launches)
    long fwd_chain_cap = 0;     // blocks of that kernel the device holds at once
    bool dinv = false;          // the factors in Lbuf carry their inverted diagonal blocks
    float* h1f = nullptr;
    float* f32 = nullptr;     // C x d_y FP32 network output
    float* d32 = nullptr;     // n_act x C x ldd32 gelu'(z), zero padded
    __hip_bfloat16* B16 = nullptr;  // C x d_y x r BF16 whitened Jacobian (at the proposal)
    // observation-space (dual) form: the state's Jacobian; the factor buffers hold the
    // Cholesky factors of I + B B^T (d_y x d_y) instead of I + H
    bool dual = false;
    int kdim = 0;                   // order of the factorised matrix: r, or d_y in the dual form
    __hip_bfloat16* Bs16 = nullptr; // C x d_y x ldb (mixed path)
    double* Bs64 = nullptr;         // C x d_y x r (FP64 path)
    // delayed acceptance (DINO_METHOD_DA_MMALA): true misfit of the states, compacted
    // full-proposal rows of the first-stage passes, true-model activations and outputs
    bool da = false;
    int rT = 0;               // true-model input width: r + the complement coordinates it reads
    double* phit = nullptr;   // C: true misfit of the states
    int64_t* passes = nullptr;// C: first-stage passes (true-model evaluations)
    int32_t* pos = nullptr;   // C: compacted row of a passing chain, -1 otherwise
    int32_t* npass = nullptr; // 1: rows in the compacted batch
    double* zin = nullptr;    // C x rT full-proposal coordinates the true model reads
    double* th0 = nullptr;    // C x wT true-model activations (FP64 path)
    double* th1 = nullptr;
    double* fT64 = nullptr;   // C x d_y true outputs (FP64 path)
    float* th0f = nullptr;    // mixed path
    float* th1f = nullptr;
    float* fT32 = nullptr;
    // delayed acceptance on a dense basis: the compacted full-proposal complement draws w+,
    // their projections U^T w+ and the chain of every compacted row
    double* wb64 = nullptr;   // C x d_m (FP64 path)
    float* wb32 = nullptr;    // C x ldz (mixed path)
    double* tp64 = nullptr;   // C x r
    float* tp32 = nullptr;    // C x r
    int32_t* rowchain = nullptr;
    // trace
    float* xtrace = nullptr;  // capacity x C x r
    double* phitrace = nullptr;
    // launch graphs: one per (chain bucket, steps) captured on cap_stream and replayed on
    // the caller's stream (steps whose kernel arguments are all fixed per problem)
    struct StepGraph {
        int n = 0, steps = 0;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<StepGraph> graphs;
    hipStream_t cap_stream = nullptr;
    int launch_mode = 1;      // DINO_LAUNCH_GRAPH
    int graph_steps = 8;      // transitions per captured graph
    // stage profiling
    bool profile = false;
    // ring of per-step stage events, drained when full and on read (no per-step host wait)
    static constexpr int PROFILE_RING = 128;
    std::vector<hipEvent_t> ev;   // PROFILE_RING x (DINO_N_STAGES + 1)
    int ring_used = 0;
    double stage_ms[DINO_N_STAGES] = {};
    int32_t stage_launches[DINO_N_STAGES] = {};
    int64_t profiled_steps = 0;
};

namespace dino {

// Tuning table (runtime.hip): the implementation chosen for a stage at a shape (a, b, c),
// process-wide; -1 when the shape has no entry (the launcher's default then applies).
enum TuneKind : int { TUNE_CHOL = 0, TUNE_FWD64 = 1, TUNE_FWD32 = 2, TUNE_HESS = 3, TUNE_FWDCHAIN = 4, TUNE_DUALSOLVE = 5 };
constexpr int CHOL_VARIANTS = 7;
int tuned_choice(int kind, int a, int b, int c);
void set_tuned_choice(int kind, int a, int b, int c, int choice, const std::vector<double>& ms);

// launch helpers (kernels_*.hip)
void launch_forward(dino_problem* p, int n, const double* x, double* f_out, hipStream_t st);
void launch_reverse_jacobian(dino_problem* p, int n, double* B_out, hipStream_t st);
void launch_misfit_grad(dino_problem* p, int n, const double* f, const double* B, double* phi, double* g,
                        hipStream_t st);
// A_c (slot-selected) = [I +] B_c^T B_c; lower tiles only unless full.
void launch_gn_hessian_slot(dino_problem* p, int n, const double* B, double* A, long strideA, const int32_t* slot,
                            int slot_xor, long slot_stride, int add_identity, int full, hipStream_t st);
// Matrices addressed per chain c as base + c*stride + (slot[c] ^ slot_xor) * slot_stride.
void launch_cholesky_slot(int n, int r, double* A, long strideA, const int32_t* slot, int slot_xor,
                          long slot_stride, double* logdet, int32_t* ok, hipStream_t st);
void launch_cholesky_variant(int variant, int n, int r, double* A, long strideA, const int32_t* slot, int slot_xor,
                             long slot_stride, double* logdet, int32_t* ok, hipStream_t st);
int cholesky_variant_max(int variant);
void launch_fill_identity(int n, int r, double* A, long strideA, const int32_t* slot, int slot_xor, long slot_stride,
                          hipStream_t st);
void launch_propose_slot(dino_problem* p, int n, const double* x, const double* g, const double* L, long strideL,
                         const int32_t* slot, int slot_xor, long slot_stride, const double* xi_given, bool use_meta,
                         double* xp, double* lfwd, const double* logdet, hipStream_t st);
// The accept kernels also end the step of each chain: trace row (the chain's step counter,
// below the trace capacity), running sums, step counter and life cycle.
void launch_accept(dino_problem* p, int n, hipStream_t st);
// Per-step bookkeeping of chains [0, n): step counters, life cycle, running sums, trace row.
// Sets the metadata of chains [c0, c0 + n) (index = first_index + c - c0) and zeroes their sums.
void launch_meta_fill(dino_problem* p, int c0, int n, uint64_t key0, uint64_t key1, int64_t budget, int64_t burn,
                      int32_t row, int32_t state, int32_t first_index, hipStream_t st);
// Posterior mean of chains [c0, c0 + n): xbar = sum_c sumx_c / (n count), field = Psi_r xbar.
void launch_request_mean(dino_problem* p, int c0, int n, int64_t count, double* xbar, double* field,
                         hipStream_t st);
void launch_log_rho(dino_problem* p, int n, const double* x, const double* phi_x, const double* g_x,
                    const double* L_x, const double* logdet_x, const double* xp, const double* phi_p,
                    const double* g_p, const double* L_p, const double* logdet_p, double* out, hipStream_t st);
// After the accept kernel of the same step (it reads the advanced step counter).
void launch_complement(dino_problem* p, int n, hipStream_t st);
// dual form (kernels_chain.hip, kernels_mfma.hip, kernels_geometry.hip)
void launch_propose_dual(dino_problem* p, int n, hipStream_t st);
void launch_accept_dual(dino_problem* p, int n, hipStream_t st);
void launch_pcn_propose(dino_problem* p, int n, hipStream_t st);
void launch_pcn_accept(dino_problem* p, int n, hipStream_t st);
void launch_mala_propose(dino_problem* p, int n, hipStream_t st);
void launch_lapcn_propose(dino_problem* p, int n, hipStream_t st);
void launch_mala_accept(dino_problem* p, int n, hipStream_t st);
// Whether the BF16 reverse sweep covers the network: it holds at most 16 row blocks of 32
// (the reduced dimension and every hidden width at most 512).
bool sweep_width_ok(const dino_ctx* ctx);
// Whether the BF16 Gauss-Newton Hessian kernel's LDS (B^T and the residual) fits one block.
bool hess_bf16_lds_fits(int r, int dy);
// Whether the dual-form transition kernels' LDS (vectors, scratch and, on the BF16 path,
// the staged B) fits one block for reduced dimension r and d_y observations.
bool dual_lds_fits(int r, int dy, bool bf16);
void launch_keep_jacobian(dino_problem* p, int n, hipStream_t st);
int jacobian_ld(const dino_problem* p);
void launch_eval_propose_dual(dino_problem* p, int n, const double* x, const double* g, const void* B,
                              const double* K, const double* logdet, const double* xi, double* xp, double* lfwd,
                              hipStream_t st);
void launch_eval_log_rho_dual(dino_problem* p, int n, const double* x, const double* phi_x, const double* g_x,
                              const void* B_x, const double* K_x, const double* logdet_x, const double* xp,
                              const double* phi_p, const double* g_p, const void* B_p, const double* K_p,
                              const double* logdet_p, double* out, hipStream_t st);
void launch_jacobian_to_double(dino_problem* p, int n, double* out, hipStream_t st);
// delayed acceptance (kernels_geometry.hip, kernels_chain.hip)
void launch_true_forward(dino_problem* p, int n, const double* zin, const int* m_dev, hipStream_t st);
// C[m][n] = sum_k A[m][k] B[n][k] (B: N x K row-major) for rows m below M (and below *m_dev
// when given): the forward layer kernels without bias or activation (kernels_geometry.hip)
void launch_gemm_nt64(int M, int K, int N, const double* A, int lda, const double* B, double* C, int ldc,
                      const int* m_dev, hipStream_t st);
void launch_gemm_nt32(int M, int K, int N, const float* A, int lda, const float* B, float* C, int ldc,
                      const int* m_dev, hipStream_t st);
void build_dense_basis_device(Basis& b, const std::vector<double>& U, const double* lam_dis);
void launch_da_gather(dino_problem* p, int n, hipStream_t st);
void launch_da_init(dino_problem* p, int n, hipStream_t st);
void launch_da_accept(dino_problem* p, int n, hipStream_t st);
void launch_true_misfit(dino_problem* p, int n, double* out, hipStream_t st);
// Also the whitened residual and the misfit phi from the FP32 output f (the mixed path has
// no separate misfit launch).
bool gram_chol_bf16_fits(int r, int dy);
void launch_gram_chol_bf16(dino_problem* p, int n, const __hip_bfloat16* B, const float* f, double* phi, double* A,
                           long strideA, const int32_t* slot, int slot_xor, long slot_stride, double* g,
                           double* logdet, int32_t* ok, int dinv, hipStream_t st);
void launch_gram_bf16(dino_problem* p, int n, const __hip_bfloat16* B, const float* f, double* phi, double* A,
                      long strideA, const int32_t* slot, int slot_xor, long slot_stride, double* g, hipStream_t st);
void launch_gram_f64(dino_problem* p, int n, const double* B, double* A, long strideA, const int32_t* slot,
                     int slot_xor, long slot_stride, hipStream_t st);
void launch_btb(dino_problem* p, int n, double* H, hipStream_t st);
void launch_init_draws(dino_problem* p, int draw_x, int draw_z, hipStream_t st);
void launch_normals(uint64_t seed, uint64_t rid, int n, int stream_id, int64_t step, int count, double* out,
                    hipStream_t st);
void launch_copy_rows(int n, int width, const double* src, double* dst, hipStream_t st);

// n_steps transitions of chains [0, n) (runtime.hip).
void run_steps(dino_problem* p, int n, int n_steps, hipStream_t st);
void release_graphs(dino_problem* p);
// Problem with n_rows request rows; serving pools keep running sums (runtime.hip).
dino_problem* create_problem(dino_ctx* ctx, const dino_problem_desc* desc, int n_rows, bool serving);
void destroy_problem(dino_problem* p);

// basis
void build_basis_device(Basis& b);
// Whitened KLE coordinates of nf fields (x: nf x r, zp: nf x (d_m - r), either may be
// null) and back; t1, t2 are nf x d_m scratch.
void launch_encode(const Basis& b, int nf, const double* fields, double* x, double* zp, double* t1, double* t2,
                   hipStream_t st);
void launch_decode(const Basis& b, int nf, const double* x, const double* zp, double* fields, double* t1, double* t2,
                   hipStream_t st);
void launch_posterior(dino_problem* p, int burn_in, double* mean, double* var, double* xbar, double* S,
                      hipStream_t st);
void launch_ess(dino_problem* p, int burn_in, double* ess, hipStream_t st);

NetView net_view(const dino_ctx* ctx);

// mixed-precision path (kernels_mfma.hip, kernels_geometry.hip)
int sweep_nmb(const dino_ctx* ctx);
// Output layer W (fan_out x fan_in) for the sweep's initial Lambda: entry
// ((mb * 4 + jq) * fan_out + i) * 8 + 4 h + t = W[i][32 mb + 8 jq + 4 h + t] (zero beyond fan_in).
void pack_sweep_wout(const std::vector<double>& W, int fan_out, int fan_in, int nmb_t, std::vector<float>& out);
void pack_sweep_tiles(const std::vector<double>& W, int fan_out, int fan_in, int nmb_t, std::vector<uint16_t>& out,
                      int& nmb_out);
// FP32 forward; the first layer reads x64 (FP64, rounded on load) if given, else xf.
void launch_forward32(dino_problem* p, int n, const float* xf, const double* x64, float* f_out, hipStream_t st);
int fwd_chain_capacity(int device);
bool fwd_chain_usable(const dino_problem* p, int n);
void launch_sweep_bf16(dino_problem* p, int n, const float* d32, int ldd, __hip_bfloat16* Bout, hipStream_t st);
// FP8 reverse sweep (kernels_fp8.hip): same output as launch_sweep_bf16, products in e4m3,
// the left operand as one e4m3 term or two (terms = 1 or 2).
void launch_sweep_fp8(dino_problem* p, int n, int terms, const float* d32, int ldd, __hip_bfloat16* Bout,
                      hipStream_t st);
// Whether the FP8 sweep holds the network for d_y observations (Lambda of 64 rows and the
// gelu' rows of its chains in one block's LDS).
bool fp8_sweep_ok(const dino_ctx* ctx, int dy);
// OCP e4m3 code of v (round to nearest even, saturating at 448).
uint8_t e4m3_encode(double v);
// FP8 W^T of a layer (from its host copy) with power-of-two column exponents.
void pack_fp8_layer(Layer& ly);
// (Re)builds ctx->fp8_layers from the loaded network's FP8 copies.
void build_fp8_table(dino_ctx* ctx);
void launch_hess_bf16(dino_problem* p, int n, const __hip_bfloat16* B, const float* f, double* phi, double* A,
                      long strideA, const int32_t* slot, int slot_xor, long slot_stride, double* g, hipStream_t st);
void launch_to_float(long count, const double* x, float* xf, hipStream_t st);
void launch_to_double(long count, const float* xf, double* x, hipStream_t st);
void launch_sym_from_lower(int n, int r, const double* A, double* H, hipStream_t st);

}  // namespace dino
