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
// Per layer: stage the gelu' rows of the block's chains in LDS; the four waves (two row
// halves by two column halves) run the products; after a barrier each lane adds the
// residual branch to its own elements and writes them back over Lambda, or, after the
// input layer, writes its rows of B scaled by Gamma^-1/2.
#include "dino_internal.hpp"

namespace dino {

typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(8))) int i32x8;
typedef __attribute__((ext_vector_type(4))) int i32x4;

constexpr int F8_ROWS = 64;        // Lambda rows per block
constexpr int F8_TPB = 256;        // 4 waves
constexpr int F8_MAX_TILES = 13;   // 32-column tiles per wave: layers up to 832 units

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

// LDS: Lambda (64 rows of ldl BF16, K padded to 64) and the gelu' rows of up to nch chains
// (ldds floats each, zero beyond the layer's K).
static int fp8_kpad(int wmax) { return (wmax + 63) / 64 * 64; }
static int fp8_nch(int dy) { return (F8_ROWS - 1) / dy + 2; }
static size_t fp8_sweep_lds(int wmax, int dy) {
    return (size_t)F8_ROWS * (fp8_kpad(wmax) + 8) * 2 + (size_t)fp8_nch(dy) * fp8_kpad(wmax) * 4;
}

// Operand layout of the 32 x 32 x 64 FP8 form (gfx950): lane (m, h) holds K = 16h .. 16h+15
// in bytes 0-15 and K = 32 + 16h .. 32 + 16h + 15 in bytes 16-31, and its scale byte
// covers the MX block K = 32h .. 32h + 31 of its row (column).
//
// The weights go through a buffer resource (byte offset voff + soff): buffer loads count
// on the vector-memory counter alone, so each product waits only for its own operands.
__device__ __forceinline__ i32x8 bload32(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
    const i32x4 lo = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0);
    const i32x4 hi = __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 32, soff, 0);
    return i32x8{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
}

// 2^-e for |e| <= 126 (exponent field arithmetic, exact).
__device__ __forceinline__ float pow2_neg(int e) { return __int_as_float((127 - e) << 23); }

// The A operand of one lane for the K chunk at kc: its 32 values v (K 16h.. and 32+16h..)
// of row lrow (Lambda, BF16) times drow (gelu', FP32), the MX block exponents of the
// chunk's two blocks (shared with the partner lane m + 32 (1 - h)), the e4m3 bytes of
// hi and, for NA = 2, of lo = rne((v 2^-e - hi) 16). sa: the lane's scale byte for hi.
template <int NA>
__device__ __forceinline__ void quantise_chunk(const __hip_bfloat16* lrow, const float* drow, int kc, int h,
                                               i32x8& ahi, i32x8& alo, int& sa) {
    float v[32];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const int k0 = kc + 32 * g + 16 * h;
        const uint4 x0 = *reinterpret_cast<const uint4*>(lrow + k0);
        const uint4 x1 = *reinterpret_cast<const uint4*>(lrow + k0 + 8);
        const float4 d0 = *reinterpret_cast<const float4*>(drow + k0);
        const float4 d1 = *reinterpret_cast<const float4*>(drow + k0 + 4);
        const float4 d2 = *reinterpret_cast<const float4*>(drow + k0 + 8);
        const float4 d3 = *reinterpret_cast<const float4*>(drow + k0 + 12);
        const unsigned xs[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
        const float ds[16] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w,
                              d2.x, d2.y, d2.z, d2.w, d3.x, d3.y, d3.z, d3.w};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            v[16 * g + 2 * j] = __uint_as_float(xs[j] << 16) * ds[2 * j];
            v[16 * g + 2 * j + 1] = __uint_as_float(xs[j] & 0xFFFF0000u) * ds[2 * j + 1];
        }
    }
    float m0 = 0.f, m1 = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        m0 = fmaxf(m0, fabsf(v[j]));
        m1 = fmaxf(m1, fabsf(v[16 + j]));
    }
    m0 = fmaxf(m0, __shfl_xor(m0, 32));
    m1 = fmaxf(m1, __shfl_xor(m1, 32));
    const int e0 = m0 > 0.f ? max(-120, min(120, ilogbf(m0) - 7)) : 0;
    const int e1 = m1 > 0.f ? max(-120, min(120, ilogbf(m1) - 7)) : 0;
    const float s0 = pow2_neg(e0), s1 = pow2_neg(e1);
    sa = 127 + (h ? e1 : e0);
#pragma unroll
    for (int j = 0; j < 32; ++j) v[j] *= (j < 16 ? s0 : s1);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        int w = 0;
        w = __builtin_amdgcn_cvt_pk_fp8_f32(v[4 * q], v[4 * q + 1], w, false);
        w = __builtin_amdgcn_cvt_pk_fp8_f32(v[4 * q + 2], v[4 * q + 3], w, true);
        ahi[q] = w;
    }
    if (NA == 2) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const auto p0 = __builtin_amdgcn_cvt_pk_f32_fp8(ahi[q], false);
            const auto p1 = __builtin_amdgcn_cvt_pk_f32_fp8(ahi[q], true);
            int w = 0;
            w = __builtin_amdgcn_cvt_pk_fp8_f32((v[4 * q] - p0[0]) * 16.f, (v[4 * q + 1] - p0[1]) * 16.f, w, false);
            w = __builtin_amdgcn_cvt_pk_fp8_f32((v[4 * q + 2] - p1[0]) * 16.f, (v[4 * q + 3] - p1[1]) * 16.f, w, true);
            alo[q] = w;
        }
    }
}

// The products of one layer for a wave with NT column tiles over the K chunks of the
// layer: A quantised from LDS one chunk ahead of the products that use it, the weights'
// first tiles of the next chunk loaded while the current chunk multiplies.
template <int NT, int NA>
__device__ __forceinline__ void fp8_products(f32x16 (&acc)[F8_MAX_TILES], const int (&sb)[F8_MAX_TILES],
                                             const __hip_bfloat16* lrow, const float* drow, int h,
                                             __amdgpu_buffer_rsrc_t wrs, int voff, int tstride, int kp) {
    constexpr int P = NT < 4 ? NT : 4;
    i32x8 bp[P];
#pragma unroll
    for (int t = 0; t < P; ++t) bp[t] = bload32(wrs, voff, t * tstride);
    i32x8 ahi, alo;
    int sa;
    quantise_chunk<NA>(lrow, drow, 0, h, ahi, alo, sa);
    for (int kc = 0; kc < kp; kc += 64) {
        i32x8 b[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) b[t] = t < P ? bp[t] : bload32(wrs, voff + kc, t * tstride);
        const int kn = min(kc + 64, kp - 64);  // a repeat of the last chunk at the end
#pragma unroll
        for (int t = 0; t < P; ++t) bp[t] = bload32(wrs, voff + kn, t * tstride);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            acc[t] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(ahi, b[t], acc[t], 0, 0, 0, sa, 0, sb[t]);
            if (NA == 2)
                acc[t] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(alo, b[t], acc[t], 0, 0, 0, sa - 4, 0, sb[t]);
        }
        quantise_chunk<NA>(lrow, drow, kn, h, ahi, alo, sa);
    }
}

template <int NA>
__global__ __launch_bounds__(F8_TPB) void jac_sweep_fp8_kernel(Fp8SweepArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __hip_bfloat16* lam = reinterpret_cast<__hip_bfloat16*>(smem);           // F8_ROWS x ldl
    float* dS = reinterpret_cast<float*>(smem + (size_t)F8_ROWS * a.ldl * 2);  // nch x ldds
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l32 = lane & 31, h = lane >> 5, wm = wave & 1, wn = wave >> 1;
    const long m0 = (long)blockIdx.x * F8_ROWS;
    const long c_first = m0 / a.dy;
    const int nchb = (int)((min(a.M, m0 + F8_ROWS) - 1) / a.dy - c_first + 1);
    // Lambda_L: row m % d_y of the output layer, zero past its width (every column is written)
    for (int e = tid; e < F8_ROWS * a.ldl; e += F8_TPB) {
        const int row = e / a.ldl, k = e - row * a.ldl;
        const long m = m0 + row;
        const float v = (m < a.M && k < a.w_out) ? a.Wout[(m % a.dy) * (long)a.w_out + k] : 0.f;
        lam[e] = __float2bfloat16(v);
    }
    const int my_row = 32 * wm + l32;
    const long my_m = m0 + my_row;
    const int my_slot = my_m < a.M ? (int)(my_m / a.dy - c_first) : 0;
    const __hip_bfloat16* lrow = lam + my_row * a.ldl;
    const float* drow = dS + my_slot * a.ldds;

    for (int li = 0; li < a.n_layers; ++li) {
        const Fp8SweepLayer L = a.layers[li];
        const float* dl = L.act >= 0 ? a.d32 + L.act * a.dstride : nullptr;
        // gelu' rows of the block's chains (ones for a linear layer), zero past K; the
        // previous layer's products and write-back are complete past this barrier
        __syncthreads();
        for (int e = tid; e < nchb * L.kp; e += F8_TPB) {
            const int c = e / L.kp, k = e - c * L.kp;
            float v = 0.f;
            if (k < L.K) v = dl ? dl[(c_first + c) * (long)a.ldd + k] : 1.f;
            dS[c * a.ldds + k] = v;
        }
        __syncthreads();
        const int ntiles = (L.N + 31) / 32;
        const int half = (ntiles + 1) / 2;
        const int t0 = wn * half;
        const int nt = min(half, ntiles - t0);
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
        const int voff = (32 * t0 + l32) * L.kp + 16 * h;
        const int tstride = 32 * L.kp;
        switch (nt) {
#define F8_CASE(NT) \
    case NT: fp8_products<NT, NA>(acc, sb, lrow, drow, h, wrs, voff, tstride, L.kp); break;
            F8_CASE(1) F8_CASE(2) F8_CASE(3) F8_CASE(4) F8_CASE(5) F8_CASE(6) F8_CASE(7)
            F8_CASE(8) F8_CASE(9) F8_CASE(10) F8_CASE(11) F8_CASE(12) F8_CASE(13)
#undef F8_CASE
            default: break;
        }
        __syncthreads();  // every wave has read Lambda for this layer
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
                const long m = m0 + row;
                if (m >= a.M) continue;
                const long c = m / a.dy;
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
                        a.B[m * a.ldb + col] = __float2bfloat16(v);
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
        if (ctx->layers[l].fan_in > 32 * F8_MAX_TILES * 2 || ctx->layers[l].fan_out > 32 * F8_MAX_TILES * 2)
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
    DINO_REQUIRE(blocks < (1L << 31), DINO_EINVAL, "too many Jacobian rows for one launch");
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
    for (int n = 0; n < fan_in; ++n) {
        double mx = 0.0;
        for (int k = 0; k < fan_out; ++k) mx = std::max(mx, std::fabs(ly.hostW[(size_t)k * fan_in + n]));
        const int e = mx > 0.0 ? std::max(-127, std::min(127, std::ilogb(mx) - 7)) : 0;
        ex[n] = (uint8_t)(127 + e);
        for (int k = 0; k < fan_out; ++k)
            wt[(size_t)n * kp + k] = e4m3_encode(std::ldexp(ly.hostW[(size_t)k * fan_in + n], -e));
    }
    ly.kp8 = kp;
    DINO_HIP(hipMalloc(&ly.WT8, wt.size() + ex.size()));
    ly.wexp8 = ly.WT8 + wt.size();
    DINO_HIP(hipMemcpy(ly.WT8, wt.data(), wt.size(), hipMemcpyHostToDevice));
    DINO_HIP(hipMemcpy(ly.wexp8, ex.data(), ex.size(), hipMemcpyHostToDevice));
}

}  // namespace dino
