// Reduced Jacobian (the surrogate Jacobian of Sec. 4, the display after eq. rb_dino) with
// FP8 products for the widest networks: the reverse sweep
//     Lambda_L = W_out,   Lambda_{l-1} = [Lambda_l +] (Lambda_l diag(gelu'(z_l))) W_l,
//     B = Gamma^-1/2 Lambda_0,
// on the gfx950 MFMA form v_mfma_scale_f32_32x32x64_f8f6f4 (OCP e4m3 operands, FP32
// accumulation, one E8M0 power-of-two scale per lane and operand).
//
// One block owns 64 rows of Lambda (row m = chain m / d_y, observed output m % d_y) for
// the whole sweep: Lambda stays in LDS in BF16 from the output layer to the input layer,
// so HBM sees only the gelu' rows, the weights (through L2) and B.
//
// Operands. The weights W_l^T are e4m3 with one power-of-two scale per output channel
// (column of W_l), packed once per network. The left operand A = Lambda diag(d) is
// quantised as the products run, by each lane for its own 64-wide K chunk, in MX blocks
// of 32 along K with the power of two that brings the block's largest magnitude into
// [128, 256) (e4m3 holds up to 448, so nothing saturates). With NA = 2 terms A is also
// split as A = hi + lo, lo the e4m3 rounding of the remainder at 16x the scale, and each
// weight operand serves two products: the rounding error of A drops from ~2^-4 to ~2^-8
// relative. That error, unlike the weights', changes from state to state, so it is what
// roughens the metric the proposal densities see (a single e4m3 term cuts mMALA's
// acceptance far below the FP64 path's at the largest shape).
//
// Per layer: stage the gelu' rows of the block's chains in LDS; the eight waves (two row
// halves by four column quarters) run the products; after a barrier each lane adds the
// residual branch to its own elements and writes them back over Lambda, or, after the
// input layer, writes its rows of B scaled by Gamma^-1/2.
#include "dino_internal.hpp"

namespace dino {

typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(8))) int i32x8;
typedef __attribute__((ext_vector_type(4))) int i32x4;

constexpr int F8_ROWS = 64;        // Lambda rows per block
constexpr int F8_TPB = 512;        // 8 waves: two per SIMD, so one's VALU work overlaps the other's products
constexpr int F8_MAX_TILES = 7;    // 32-column tiles per wave (a quarter of the layer): layers up to 896 units

struct Fp8SweepArgs {
    long M;                       // rows: chains x d_y
    int dy, n_layers, ldd, ldl, ldds, nch, ldb, w_out;
    long dstride;                 // gelu' rows of activated layer a start at d32 + a dstride
    const float* d32;
    const Fp8SweepLayer* layers;  // device table, processing order
    const float* Wout;            // output layer (d_out x w_out, FP32): Lambda_L rows
    const double* winv;           // Gamma^-1/2 per request row (rows x d_y)
    const int32_t* rows;          // request row per chain, or null
    __hip_bfloat16* B;            // (chains x d_y) x ldb
};

// LDS: Lambda (64 rows of ldl BF16, K padded to 64), the gelu' rows of up to nch chains
// (ldds floats each, zero beyond the layer's K) and the staged left operand.
static int fp8_kpad(int wmax) { return (wmax + 63) / 64 * 64; }
static int fp8_nch(int dy) { return (F8_ROWS - 1) / dy + 2; }
static size_t fp8_sweep_lds(int wmax, int dy);

// Operand layout of the 32 x 32 x 64 FP8 form (gfx950): lane (m, h) holds K = 16h .. 16h+15
// in bytes 0-15 and K = 32 + 16h .. 32 + 16h + 15 in bytes 16-31, and its scale byte
// covers the MX block K = 32h .. 32h + 31 of its row (column).
//
// The weights are packed in operand order: for each 32-column tile and 64-deep K chunk,
// 2 KB = two halves of 64 lanes x 16 bytes (half 0: K 16h .. 16h + 15 of the lane's
// column, half 1: K 32 + 16h ..), so each load instruction of a wave reads 1 KB of
// contiguous memory. They go through a buffer resource (byte offset voff + soff): buffer
// loads count on the vector-memory counter alone, so each product waits only for its own
// operands.
__device__ __forceinline__ i32x8 bload32(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
    const i32x4 lo = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0);
    const i32x4 hi = __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 1024, soff, 0);
    return i32x8{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
}

// 2^-e for |e| <= 126 (exponent field arithmetic, exact).
__device__ __forceinline__ float pow2_neg(int e) { return __int_as_float((127 - e) << 23); }

// Staging of the quantised left operand: two buffers (chunk parity) of 64 rows; a row
// holds hi (64 bytes, the chunk's K in natural order), lo (64 bytes) and padding, and the
// scale bytes of its two MX blocks (hi's; lo's is 4 less).
constexpr int F8_QP = 144;                       // bytes per staged row
constexpr int F8_QBUF = F8_ROWS * F8_QP;         // one parity
constexpr int F8_QLDS = 2 * F8_QBUF + 2 * F8_ROWS * 2;

static size_t fp8_sweep_lds(int wmax, int dy) {
    return (size_t)F8_ROWS * (fp8_kpad(wmax) + 8) * 2 + (size_t)fp8_nch(dy) * fp8_kpad(wmax) * 4 + F8_QLDS;
}

// One lane's share of quantising a K chunk: 8 values of row qrow (Lambda, BF16) at
// K = kc + 32 b + 8 q .. + 7 times the gelu' row qd; the lanes lane ^ 1, ^ 2, ^ 3 hold
// the rest of the MX block. Writes the hi (and, NA = 2, lo) e4m3 bytes and, from the
// q = 0 lane, the block's scale byte.
template <int NA>
__device__ __forceinline__ void quantise_share(const __hip_bfloat16* qrow, const float* qd, int kc, int b, int q,
                                               uint8_t* qdst, uint8_t* qsc) {
    const int k0 = kc + 32 * b + 8 * q;
    const uint4 x = *reinterpret_cast<const uint4*>(qrow + k0);
    const float4 d0 = *reinterpret_cast<const float4*>(qd + k0);
    const float4 d1 = *reinterpret_cast<const float4*>(qd + k0 + 4);
    const unsigned xs[4] = {x.x, x.y, x.z, x.w};
    const float ds[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
    float v[8];
    float m = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        v[2 * j] = __uint_as_float(xs[j] << 16) * ds[2 * j];
        v[2 * j + 1] = __uint_as_float(xs[j] & 0xFFFF0000u) * ds[2 * j + 1];
        m = fmaxf(m, fmaxf(fabsf(v[2 * j]), fabsf(v[2 * j + 1])));
    }
    m = fmaxf(m, __shfl_xor(m, 1));
    m = fmaxf(m, __shfl_xor(m, 2));
    const int e = m > 0.f ? max(-120, min(120, ilogbf(m) - 7)) : 0;
    const float sc = pow2_neg(e);
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] *= sc;
    int hi[2];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        int t = 0;
        t = __builtin_amdgcn_cvt_pk_fp8_f32(v[4 * w], v[4 * w + 1], t, false);
        t = __builtin_amdgcn_cvt_pk_fp8_f32(v[4 * w + 2], v[4 * w + 3], t, true);
        hi[w] = t;
    }
    *reinterpret_cast<int2*>(qdst + 32 * b + 8 * q) = make_int2(hi[0], hi[1]);
    if (NA == 2) {
        int lo[2];
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const auto p0 = __builtin_amdgcn_cvt_pk_f32_fp8(hi[w], false);
            const auto p1 = __builtin_amdgcn_cvt_pk_f32_fp8(hi[w], true);
            int t = 0;
            t = __builtin_amdgcn_cvt_pk_fp8_f32((v[4 * w] - p0[0]) * 16.f, (v[4 * w + 1] - p0[1]) * 16.f, t, false);
            t = __builtin_amdgcn_cvt_pk_fp8_f32((v[4 * w + 2] - p1[0]) * 16.f, (v[4 * w + 3] - p1[1]) * 16.f, t,
                                                true);
            lo[w] = t;
        }
        *reinterpret_cast<int2*>(qdst + 64 + 32 * b + 8 * q) = make_int2(lo[0], lo[1]);
    }
    if (q == 0) qsc[b] = (uint8_t)(127 + e);
}

// The products of one layer for a wave with NT column tiles (NT = 0: the wave only takes
// its share of the quantisation). Chunk i multiplies the operand staged in parity i % 2
// while the block quantises chunk i + 1 into the other parity (the last chunk quantises a
// repeat of itself there, which nothing reads: that parity's readers passed the previous
// barrier); one barrier per chunk. The weights' first tiles of the next chunk load while
// the current chunk multiplies.
template <int NT, int NA>
__device__ __forceinline__ void fp8_products(f32x16 (&acc)[F8_MAX_TILES], const int (&sb)[F8_MAX_TILES],
                                             uint8_t* qlds, int my_row, int h,
                                             const __hip_bfloat16* qrow, const float* qd, int qr, int qb, int qq,
                                             __amdgpu_buffer_rsrc_t wrs, int voff, int tstride, int kp) {
    constexpr int P = NT < 2 ? NT : 2;
    i32x8 bp[P > 0 ? P : 1];
#pragma unroll
    for (int t = 0; t < P; ++t) bp[t] = bload32(wrs, voff, t * tstride);
    uint8_t* qsc = qlds + 2 * F8_QBUF;  // [parity][row][block]
    quantise_share<NA>(qrow, qd, 0, qb, qq, qlds + qr * F8_QP, qsc + qr * 2);
    __syncthreads();
    const int nchunk = kp / 64;
    for (int i = 0; i < nchunk; ++i) {
        const int kc = 64 * i, par = i & 1;
        const int kn = min(kc + 64, kp - 64);  // the next chunk (a repeat of the last one at the end)
        if (NT > 0) {
            const uint8_t* arow = qlds + par * F8_QBUF + my_row * F8_QP + 16 * h;
            const uint4 h0 = *reinterpret_cast<const uint4*>(arow);
            const uint4 h1 = *reinterpret_cast<const uint4*>(arow + 32);
            const i32x8 ahi = {(int)h0.x, (int)h0.y, (int)h0.z, (int)h0.w, (int)h1.x, (int)h1.y, (int)h1.z, (int)h1.w};
            i32x8 alo = ahi;
            if (NA == 2) {
                const uint4 l0 = *reinterpret_cast<const uint4*>(arow + 64);
                const uint4 l1 = *reinterpret_cast<const uint4*>(arow + 96);
                alo = i32x8{(int)l0.x, (int)l0.y, (int)l0.z, (int)l0.w, (int)l1.x, (int)l1.y, (int)l1.z, (int)l1.w};
            }
            const int sa = qsc[par * F8_ROWS * 2 + my_row * 2 + h];
            i32x8 b[NT > 0 ? NT : 1];
#pragma unroll
            for (int t = 0; t < NT; ++t) b[t] = t < P ? bp[t] : bload32(wrs, voff + 32 * kc, t * tstride);
#pragma unroll
            for (int t = 0; t < P; ++t) bp[t] = bload32(wrs, voff + 32 * kn, t * tstride);
            quantise_share<NA>(qrow, qd, kn, qb, qq, qlds + (par ^ 1) * F8_QBUF + qr * F8_QP,
                               qsc + (par ^ 1) * F8_ROWS * 2 + qr * 2);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                acc[t] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(ahi, b[t], acc[t], 0, 0, 0, sa, 0, sb[t]);
                if (NA == 2)
                    acc[t] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(alo, b[t], acc[t], 0, 0, 0, sa - 4, 0,
                                                                             sb[t]);
            }
        } else {
            quantise_share<NA>(qrow, qd, kn, qb, qq, qlds + (par ^ 1) * F8_QBUF + qr * F8_QP,
                               qsc + (par ^ 1) * F8_ROWS * 2 + qr * 2);
        }
        __syncthreads();
    }
}

template <int NA>
__global__ __launch_bounds__(F8_TPB) void jac_sweep_fp8_kernel(Fp8SweepArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __hip_bfloat16* lam = reinterpret_cast<__hip_bfloat16*>(smem);           // F8_ROWS x ldl
    float* dS = reinterpret_cast<float*>(smem + (size_t)F8_ROWS * a.ldl * 2);  // nch x ldds
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l32 = lane & 31, h = lane >> 5, wm = wave & 1, wn = wave >> 1;  // wn: column quarter
    // row indices fit 32 bits (M < 2^31, checked by the launcher)
    const int M = (int)a.M;
    const int m0 = blockIdx.x * F8_ROWS;
    const int c_first = m0 / a.dy;
    const int nchb = (min(M, m0 + F8_ROWS) - 1) / a.dy - c_first + 1;
    // Lambda_L: row m % d_y of the output layer, zero past its width (every column is
    // written); one row per wave at a time, so the row's index arithmetic is uniform
    for (int row = wave; row < F8_ROWS; row += F8_TPB / 64) {
        const int m = m0 + row;
        const bool ok = m < M;
        const float* src = a.Wout + (long)(ok ? m % a.dy : 0) * a.w_out;
        for (int k = lane; k < a.ldl; k += 64)
            lam[row * a.ldl + k] = __float2bfloat16((ok && k < a.w_out) ? src[k] : 0.f);
    }
    uint8_t* qlds = smem + (size_t)F8_ROWS * a.ldl * 2 + (size_t)a.nch * a.ldds * 4;
    const int my_row = 32 * wm + l32;
    // quantiser duty: row 8 wave + lane / 8, MX block (lane / 4) % 2, quarter lane % 4
    const int qr = 8 * wave + (lane >> 3), qb = (lane >> 2) & 1, qq = lane & 3;
    const int q_m = m0 + qr;
    const int q_slot = q_m < M ? q_m / a.dy - c_first : 0;
    const __hip_bfloat16* qrow = lam + qr * a.ldl;
    const float* qd = dS + q_slot * a.ldds;

    for (int li = 0; li < a.n_layers; ++li) {
        const Fp8SweepLayer L = a.layers[li];
        const float* dl = L.act >= 0 ? a.d32 + L.act * a.dstride : nullptr;
        // gelu' rows of the block's chains (ones for a linear layer), zero past K; the
        // previous layer's products and write-back are complete past this barrier
        __syncthreads();
        for (int c = 0; c < nchb; ++c) {
            const float* src = dl ? dl + (long)(c_first + c) * a.ldd : nullptr;
            for (int k = 4 * tid; k < L.kp; k += 4 * F8_TPB) {
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (k + 4 <= L.K) {
                    v = src ? *reinterpret_cast<const float4*>(src + k) : make_float4(1.f, 1.f, 1.f, 1.f);
                } else {
                    float t[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) t[j] = k + j < L.K ? (src ? src[k + j] : 1.f) : 0.f;
                    v = make_float4(t[0], t[1], t[2], t[3]);
                }
                *reinterpret_cast<float4*>(dS + c * a.ldds + k) = v;
            }
        }
        __syncthreads();
        const int ntiles = (L.N + 31) / 32;
        const int t0 = wn * ntiles / 4;
        const int nt = (wn + 1) * ntiles / 4 - t0;
        f32x16 acc[F8_MAX_TILES];
        int sb[F8_MAX_TILES];
#pragma unroll
        for (int t = 0; t < F8_MAX_TILES; ++t) {
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[t][q] = 0.f;
            sb[t] = t < nt ? (int)L.wexp[32 * (t0 + t) + l32] : 127;  // rows padded to 32
        }
        // W^T rows are padded with zeros to a multiple of 32, so every lane of a tile reads
        // in bounds; the layer's fields are uniform (readfirstlane keeps the resource scalar)
        const uint64_t wt = (uint64_t)(uintptr_t)L.WT;
        uint8_t* wt_s = (uint8_t*)(uintptr_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(wt >> 32)) << 32) |
                                              (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)wt));
        const __amdgpu_buffer_rsrc_t wrs = __builtin_amdgcn_make_buffer_rsrc(
            wt_s, 0, __builtin_amdgcn_readfirstlane(L.rows * L.kp), 0x00020000);
        const int tstride = 32 * L.kp;            // bytes per 32-column tile
        const int voff = t0 * tstride + 16 * lane;
        switch (nt) {
#define F8_CASE(NT) \
    case NT: fp8_products<NT, NA>(acc, sb, qlds, my_row, h, qrow, qd, qr, qb, qq, wrs, voff, tstride, L.kp); break;
            F8_CASE(1) F8_CASE(2) F8_CASE(3) F8_CASE(4) F8_CASE(5) F8_CASE(6) F8_CASE(7)
            default: F8_CASE(0)
#undef F8_CASE
        }
        // past the last chunk's barrier every wave has read Lambda for this layer
        // residual branch and write-back; D register q of a tile holds row
        // 8 (q / 4) + 4 h + q % 4 of the wave's 32 rows, column l32 of the tile
        if (li + 1 < a.n_layers) {
#pragma unroll
            for (int t = 0; t < F8_MAX_TILES; ++t) {
                const int col = 32 * (t0 + t) + l32;
                if (t < nt && col < L.N) {
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        __hip_bfloat16* e = lam + (32 * wm + 8 * (q >> 2) + 4 * h + (q & 3)) * a.ldl + col;
                        const float v = acc[t][q] + (L.resid ? __bfloat162float(*e) : 0.f);
                        *e = __float2bfloat16(v);
                    }
                }
            }
        } else {
            // B = Gamma^-1/2 Lambda_0, columns up to ldb (zero beyond N)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int row = 32 * wm + 8 * (q >> 2) + 4 * h + (q & 3);
                const int m = m0 + row;
                if (m >= M) continue;
                const int c = m / a.dy;
                const long rq = a.rows ? a.rows[c] : 0;
                const double wv = a.winv[rq * a.dy + (m - c * a.dy)];
#pragma unroll
                for (int t = 0; t < F8_MAX_TILES; ++t) {
                    const int col = 32 * (t0 + t) + l32;
                    if (t < nt && col < a.ldb) {
                        float v = 0.f;
                        if (col < L.N)
                            v = (float)((double)(acc[t][q] + (L.resid ? __bfloat162float(lam[row * a.ldl + col]) : 0.f)) *
                                        wv);
                        a.B[(long)m * a.ldb + col] = __float2bfloat16(v);
                    }
                }
            }
        }
    }
}

bool fp8_sweep_ok(const dino_ctx* ctx, int dy) {
    const int L = (int)ctx->layers.size();
    if (L < 2 || !ctx->fp8_layers || dy < 1) return false;
    for (int l = 0; l < L - 1; ++l)
        if (ctx->layers[l].fan_in > 32 * F8_MAX_TILES * 4 || ctx->layers[l].fan_out > 32 * F8_MAX_TILES * 4)
            return false;
    return fp8_sweep_lds(ctx->max_width, dy) <= 160 * 1024 - 64;
}

void build_fp8_table(dino_ctx* ctx) {
    const int L = (int)ctx->layers.size();
    std::vector<Fp8SweepLayer> tab;
    int act = ctx->n_act;
    for (int l = L - 2; l >= 0; --l) {
        const Layer& ly = ctx->layers[l];
        Fp8SweepLayer s{};
        s.WT = ly.WT8;
        s.wexp = ly.wexp8;
        s.K = ly.fan_out;
        s.N = ly.fan_in;
        s.kp = ly.kp8;
        s.resid = ly.kind == DINO_LAYER_RESID ? 1 : 0;
        s.act = ly.kind != DINO_LAYER_LINEAR ? --act : -1;
        s.rows = (ly.fan_in + 31) / 32 * 32;
        tab.push_back(s);
    }
    if (ctx->fp8_layers) (void)hipFree(ctx->fp8_layers);
    ctx->fp8_layers = nullptr;
    if (tab.empty()) return;
    DINO_HIP(hipMalloc(&ctx->fp8_layers, sizeof(Fp8SweepLayer) * tab.size()));
    DINO_HIP(hipMemcpy(ctx->fp8_layers, tab.data(), sizeof(Fp8SweepLayer) * tab.size(), hipMemcpyHostToDevice));
}

void launch_sweep_fp8(dino_problem* p, int n, int terms, const float* d32, int ldd, __hip_bfloat16* Bout,
                      hipStream_t st) {
    const dino_ctx* ctx = p->ctx;
    const int L = (int)ctx->layers.size();
    DINO_REQUIRE(fp8_sweep_ok(ctx, p->d_y), DINO_EINVAL, "network too wide for the FP8 sweep");
    DINO_REQUIRE(ldd >= ctx->max_width, DINO_EINVAL, "gelu' rows shorter than the widest layer");
    DINO_REQUIRE(terms == 1 || terms == 2, DINO_EINVAL, "the FP8 sweep splits A into one or two terms");
    Fp8SweepArgs a{};
    a.M = (long)n * p->d_y;
    a.dy = p->d_y;
    a.n_layers = L - 1;
    a.ldd = ldd;
    a.ldl = fp8_kpad(ctx->max_width) + 8;
    a.ldds = fp8_kpad(ctx->max_width);
    a.nch = fp8_nch(p->d_y);
    a.ldb = jacobian_ld(p);
    a.w_out = ctx->layers[L - 1].fan_in;
    a.dstride = (long)p->C * ldd;
    a.d32 = d32;
    a.layers = ctx->fp8_layers;
    a.Wout = ctx->layers[L - 1].W32;
    a.winv = p->winv;
    a.rows = p->meta.row;
    a.B = Bout;
    const size_t lds = fp8_sweep_lds(ctx->max_width, p->d_y);
    static bool attr = false;
    if (!attr) {
        DINO_HIP(hipFuncSetAttribute((const void*)jac_sweep_fp8_kernel<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     160 * 1024 - 64));
        DINO_HIP(hipFuncSetAttribute((const void*)jac_sweep_fp8_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     160 * 1024 - 64));
        attr = true;
    }
    const long blocks = (a.M + F8_ROWS - 1) / F8_ROWS;
    DINO_REQUIRE(a.M + F8_ROWS < (1L << 31), DINO_EINVAL, "too many Jacobian rows for one launch");
    if (blocks > 0) {
        if (terms == 2)
            hipLaunchKernelGGL(jac_sweep_fp8_kernel<2>, dim3((unsigned)blocks), dim3(F8_TPB), lds, st, a);
        else
            hipLaunchKernelGGL(jac_sweep_fp8_kernel<1>, dim3((unsigned)blocks), dim3(F8_TPB), lds, st, a);
    }
    DINO_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------------
// Host side: OCP e4m3 (finite maximum 448, no infinities, 0x7f the NaN) by round to
// nearest even, and the per-network packing of W_l^T with power-of-two column exponents.

uint8_t e4m3_encode(double v) {
    const uint8_t sign = std::signbit(v) ? 0x80 : 0x00;
    const double a = std::fabs(v);
    if (std::isnan(a)) return 0x7f;
    if (a >= 464.0) return sign | 0x7e;  // beyond the midpoint of 448 and the NaN code: saturate
    if (a >= std::ldexp(1.0, -6)) {      // normal: (1 + m/8) 2^(E - 7), E = 1..15
        int e = std::ilogb(a);
        double m = std::nearbyint((a / std::ldexp(1.0, e) - 1.0) * 8.0);
        if (m == 8.0) {
            m = 0.0;
            ++e;
        }
        const int E = e + 7;
        if (E > 15 || (E == 15 && m > 6.0)) return sign | 0x7e;
        return sign | (uint8_t)(E << 3) | (uint8_t)m;
    }
    const double m = std::nearbyint(a * 512.0);  // subnormal: (m/8) 2^-6
    if (m >= 8.0) return sign | 0x08;             // rounds up to the smallest normal
    return sign | (uint8_t)m;
}

void pack_fp8_layer(Layer& ly) {
    const int fan_out = ly.fan_out, fan_in = ly.fan_in;
    const int kp = (fan_out + 63) / 64 * 64;
    const int rows = (fan_in + 31) / 32 * 32;  // zero rows up to a multiple of 32, exponent 2^0
    std::vector<uint8_t> wt((size_t)rows * kp, 0), ex(rows, 127);
    const int nchunk = kp / 64;
    for (int n = 0; n < fan_in; ++n) {
        double mx = 0.0;
        for (int k = 0; k < fan_out; ++k) mx = std::max(mx, std::fabs(ly.hostW[(size_t)k * fan_in + n]));
        const int e = mx > 0.0 ? std::max(-127, std::min(127, std::ilogb(mx) - 7)) : 0;
        ex[n] = (uint8_t)(127 + e);
        // operand order: tile n / 32, chunk k / 64, half, lane (n % 32) + 32 h, byte
        const int tile = n / 32, col = n % 32;
        for (int k = 0; k < fan_out; ++k) {
            const int c = k / 64, kk = k % 64;
            const int half = kk / 32, hh = (kk % 32) / 16, byte = kk % 16;
            const size_t off = (((size_t)tile * nchunk + c) * 2 + half) * 1024 + (size_t)(col + 32 * hh) * 16 + byte;
            wt[off] = e4m3_encode(std::ldexp(ly.hostW[(size_t)k * fan_in + n], -e));
        }
    }
    ly.kp8 = kp;
    DINO_HIP(hipMalloc(&ly.WT8, wt.size() + ex.size()));
    ly.wexp8 = ly.WT8 + wt.size();
    DINO_HIP(hipMemcpy(ly.WT8, wt.data(), wt.size(), hipMemcpyHostToDevice));
    DINO_HIP(hipMemcpy(ly.wexp8, ex.data(), ex.size(), hipMemcpyHostToDevice));
}

}  // namespace dino
