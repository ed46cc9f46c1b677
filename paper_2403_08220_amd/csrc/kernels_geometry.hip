// Surrogate forward, reduced Jacobian (reverse mode) and the reduced misfit,
// ppg and Gauss-Newton Hessian (Sec. 4 eq. rb_dino and the reduced Jacobian;
// Sec. 5.1 eqs. surrogate_rppg, surrogate_rppgnh) - FP64 path kernels.
#include "dino_internal.hpp"

namespace dino {

template <typename T>
__device__ __forceinline__ T gelu_t(T z);
template <>
__device__ __forceinline__ double gelu_t<double>(double z) {
    return 0.5 * z * (1.0 + erf(z * 0.70710678118654752440));
}
template <>
__device__ __forceinline__ float gelu_t<float>(float z) {
    return 0.5f * z * (1.0f + erff(z * 0.70710678f));
}
template <typename T>
__device__ __forceinline__ T gelu_prime_t(T z);
template <>
__device__ __forceinline__ double gelu_prime_t<double>(double z) {
    return 0.5 * (1.0 + erf(z * 0.70710678118654752440)) + z * 0.39894228040143267794 * exp(-0.5 * z * z);
}
template <>
__device__ __forceinline__ float gelu_prime_t<float>(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678f)) + z * 0.39894228f * expf(-0.5f * z * z);
}

// ---------------------------------------------------------------------------------
// Forward layer: out[m][n] = epi(sum_k in[m][k] W[n][k] + b[n]).
// Tile (16 TM rows) x (16 TN outputs) x 16 (k); 256 threads, TM x TN outputs each at
// rows ty + 16 i, columns tx + 16 j. The launcher picks the tile so that a small
// batch of chains still fills the GPU.
// m_dev (optional): a device count of the rows that hold input; blocks whose rows all lie
// at or beyond it return at once (the grid still covers M rows).
template <typename T, int TM, int TN>
__global__ __launch_bounds__(256) void fwd_layer_kernel(int M, int K, int N, const T* __restrict__ in, int ldin,
                                                        const T* __restrict__ W, const T* __restrict__ b,
                                                        int kind, T* __restrict__ out, int ldout,
                                                        T* __restrict__ dprime, int ldd, const int* m_dev) {
    constexpr int BM = 16 * TM, BN = 16 * TN;
    __shared__ T As[16][BM + 1];
    __shared__ T Ws[16][BN + 1];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    if (m_dev && m0 >= *m_dev) return;
    T acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = T(0);
    for (int k0 = 0; k0 < K; k0 += 16) {
        const int k = k0 + tx;
#pragma unroll
        for (int q = 0; q < TM; ++q) {
            const int row = ty + 16 * q;
            As[tx][row] = (m0 + row < M && k < K) ? in[(long)(m0 + row) * ldin + k] : T(0);
        }
#pragma unroll
        for (int q = 0; q < TN; ++q) {
            const int row = ty + 16 * q;
            Ws[tx][row] = (n0 + row < N && k < K) ? W[(long)(n0 + row) * K + k] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            T a[TM], w[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < TN; ++j) w[j] = Ws[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] += a[i] * w[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int m = m0 + ty + 16 * i;
        if (m >= M) continue;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int n = n0 + tx + 16 * j;
            if (n >= N) continue;
            const T z = acc[i][j] + (b ? b[n] : T(0));
            T o;
            if (kind == DINO_LAYER_LINEAR) {
                o = z;
            } else {
                o = gelu_t<T>(z);
                if (kind == DINO_LAYER_RESID) o += in[(long)m * ldin + n];
                if (dprime) dprime[(long)m * ldd + n] = gelu_prime_t<T>(z);
            }
            out[(long)m * ldout + n] = o;
        }
    }
}

// ---------------------------------------------------------------------------------
// Reverse sweep layer on rows R = (chain, output): out[R][n] = (resid ? lam[R][n] : 0)
//   + sum_k lam[R][k] * (d ? d[R / dy][k] : 1) * W[k][n],  W of shape K x N (fan_out x fan_in).
template <typename T, bool STRIDE>
__global__ __launch_bounds__(256) void rev_layer_kernel(int M, int K, int N, int dy, const T* __restrict__ lam,
                                                        int ldl, const T* __restrict__ d, int ldd,
                                                        const T* __restrict__ W, int resid, T* __restrict__ out,
                                                        int ldo) {
    __shared__ T As[16][64 + 1];
    __shared__ T Bs[16][64 + 1];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int n0 = blockIdx.x * 64;
    // STRIDE: more row tiles than the grid's y extent, tiles m0 = 64 (blockIdx.y + k gridDim.y)
    auto tile = [&](const int m0) {
        T acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = T(0);
        for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = ty + 16 * q, k = k0 + tx;
                T v = T(0);
                if (m0 + row < M && k < K) {
                    v = lam[(long)(m0 + row) * ldl + k];
                    if (d) v *= d[(long)((m0 + row) / dy) * ldd + k];
                }
                As[tx][row] = v;
                // B tile: 16 k-rows x 64 n-columns, thread t -> k = t / 64 + 4 q, n = t % 64
                const int kb = (tid >> 6) + 4 * q, nb = tid & 63;
                Bs[kb][nb] = (k0 + kb < K && n0 + nb < N) ? W[(long)(k0 + kb) * N + n0 + nb] : T(0);
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                T a[4], w[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
                for (int j = 0; j < 4; ++j) w[j] = Bs[kk][tx + 16 * j];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * w[j];
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = m0 + ty + 16 * i;
            if (m >= M) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int n = n0 + tx + 16 * j;
                if (n >= N) continue;
                T o = acc[i][j];
                if (resid) o += lam[(long)m * ldl + n];
                out[(long)m * ldo + n] = o;
            }
        }
    };
    if constexpr (STRIDE) {
        for (int m0 = blockIdx.y * 64; m0 < M; m0 += gridDim.y * 64) tile(m0);
    } else {
        tile(blockIdx.y * 64);
    }
}

// Lambda_L = diag(winv) W_out[:dy, :] for every chain: rows (c, i).
template <typename T>
__global__ void rev_init_kernel(int n, int dy, int w, const T* __restrict__ Wout, const double* __restrict__ winv,
                                const int32_t* __restrict__ rows, T* __restrict__ lam, int ldl) {
    const long total = (long)n * dy * w;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int k = (int)(e % w);
        const long R = e / w;
        const int i = (int)(R % dy);
        const long row = rows ? rows[R / dy] : 0;
        lam[R * ldl + k] = (T)(winv[row * dy + i]) * Wout[(long)i * w + k];
    }
}

// ---------------------------------------------------------------------------------
// Misfit and reduced ppg per chain: e = winv (f - y), phi = |e|^2 / 2, g = B^T e.
__global__ __launch_bounds__(256) void misfit_grad_kernel(int n, int dy, int r, const double* __restrict__ f,
                                                          const double* __restrict__ y_rows,
                                                          const double* __restrict__ winv_rows,
                                                          const int32_t* __restrict__ rows,
                                                          const double* __restrict__ B, double* __restrict__ phi,
                                                          double* __restrict__ g) {
    __shared__ double e[1024];
    __shared__ double red[4];
    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    const long row = rows ? rows[c] : 0;
    const double* y = y_rows + row * dy;
    const double* winv = winv_rows + row * dy;
    double part = 0.0;
    for (int i = tid; i < dy; i += blockDim.x) {
        const double w = winv[i];
        const double v = (w == 0.0) ? 0.0 : (f[(long)c * dy + i] - y[i]) * w;
        e[i] = v;
        part += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if ((tid & 63) == 0) red[tid >> 6] = part;
    __syncthreads();
    if (tid == 0) phi[c] = 0.5 * (red[0] + red[1] + red[2] + red[3]);
    const double* Bc = B + (long)c * dy * r;
    for (int j = tid; j < r; j += blockDim.x) {
        double acc = 0.0;
        for (int i = 0; i < dy; ++i) acc += Bc[(long)i * r + j] * e[i];
        g[(long)c * r + j] = acc;
    }
}

// ---------------------------------------------------------------------------------
// A_c = I + B_c^T B_c (or B_c^T B_c): tile 32 x 32 of the r x r output per block.
template <bool STRIDE>
__global__ __launch_bounds__(256) void gn_hessian_kernel(int n, int dy, int r, const double* __restrict__ B, double* A,
                                                         long strideA, const int32_t* __restrict__ slot,
                                                         int slot_xor, long slot_stride, int add_identity,
                                                         int full) {
    __shared__ double Bj[16][33];
    __shared__ double Bk[16][33];
    const int j0 = blockIdx.y * 32, k0 = blockIdx.x * 32;
    if (!full && k0 > j0 + 31) return;  // upper tiles: not needed by the lower Cholesky
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    // STRIDE: more chains than the grid's z extent, chains c = blockIdx.z + k gridDim.z
    auto chain = [&](const int c) {
        const double* Bc = B + (long)c * dy * r;
        double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
        for (int i0 = 0; i0 < dy; i0 += 16) {
            for (int e = tid; e < 16 * 32; e += 256) {
                const int ii = e >> 5, jj = e & 31;
                const bool okr = i0 + ii < dy;
                Bj[ii][jj] = (okr && j0 + jj < r) ? Bc[(long)(i0 + ii) * r + j0 + jj] : 0.0;
                Bk[ii][jj] = (okr && k0 + jj < r) ? Bc[(long)(i0 + ii) * r + k0 + jj] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int ii = 0; ii < 16; ++ii) {
                const double a0 = Bj[ii][ty], a1 = Bj[ii][ty + 16];
                const double b0 = Bk[ii][tx], b1 = Bk[ii][tx + 16];
                acc[0][0] += a0 * b0;
                acc[0][1] += a0 * b1;
                acc[1][0] += a1 * b0;
                acc[1][1] += a1 * b1;
            }
            __syncthreads();
        }
        const long off = (long)c * strideA + (slot ? (long)(slot[c] ^ slot_xor) * slot_stride : 0);
        double* Ac = A + off;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int j = j0 + ty + 16 * a, k = k0 + tx + 16 * b;
                if (j < r && k < r) Ac[(long)j * r + k] = acc[a][b] + ((add_identity && j == k) ? 1.0 : 0.0);
            }
    };
    if constexpr (STRIDE) {
        for (int c = blockIdx.z; c < n; c += gridDim.z) chain(c);
    } else {
        chain(blockIdx.z);
    }
}

// ---------------------------------------------------------------------------------
// Host launchers.
static inline dim3 grid2(int M, int N) { return dim3((N + 63) / 64, grid_y((M + 63) / 64)); }

// One forward layer with the largest tile that still gives >= 1024 blocks.
// FP32 layer on MFMA (v_mfma_f32_32x32x2_f32: FP32 products, FP32 accumulation): a
// block forms a 32 x 32 output tile (rows = chains, columns = outputs), its four waves
// splitting K in chunks of 8 and the partial tiles summed through LDS. Within a chunk
// of 8, lane (i, h) holds the inputs k = 8 t + 4 h + e (e < 4) for the four MFMAs
// e = 0..3 (float4 loads of A rows and W rows); A and W use the same k order, so the
// products pair up. The output layout: lane (j, h), register q holds row
// 8 (q / 4) + 4 h + q % 4 and column j of the tile.
typedef __attribute__((ext_vector_type(16))) float f32x16g;

typedef __attribute__((ext_vector_type(4))) float f32x4g;

// One 32 x 32 output tile (rows m0.., columns n0..) of an FP32 layer on the block's four
// waves. red: the block's split-K reduction buffer. wait(): called by every thread once
// the tile's weight loads are issued and before any input row is read (a no-op for a
// layer launched on its own). COH: the input rows come from other blocks of the same
// launch and are read with device-coherent loads (sc1: past any stale L1 / L2 copy);
// coh_out: the outputs are written with device-coherent stores. poison: write NaN in
// place of the outputs (a producer tile was not seen in time).
template <bool COH, typename Wait>
__device__ __forceinline__ void fwd_tile(int M, int K, int N, const float* __restrict__ in, int ldin,
                                         const double* __restrict__ in64, const float* __restrict__ W,
                                         const float* __restrict__ b, int kind, float* __restrict__ out, int ldout,
                                         float* __restrict__ dprime, int ldd, int m0, int n0, float (*red)[64][17],
                                         Wait&& wait, bool coh_out, const int& poison) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l32 = lane & 31, h = lane >> 5;
    const int arow = m0 + l32, wrow = n0 + l32;
    const bool aok = arow < M, wok = wrow < N;
    const float* ap = in64 ? nullptr : in + (long)(aok ? arow : 0) * ldin;
    const double* ap64 = in64 ? in64 + (long)(aok ? arow : 0) * ldin : nullptr;
    const float* wp = W + (long)(wok ? wrow : 0) * K;
    const bool vec = ((ldin & 3) == 0) && ((K & 3) == 0);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)in, (short)0, COH ? M * ldin * 4 : 0, 0x00020000);
    f32x16g acc;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.f;
    const int nchunk = (K + 7) / 8;
    auto coh_ld = [&](int k) { return __hip_atomic_load(ap + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
    auto load_a = [&](int t, float4& a4) {
        const int k = 8 * t + 4 * h;
        // whole chunks read rows past M as row 0 (their products only reach output rows
        // that are never stored), so the loaded values need no select
        if (vec && k + 3 < K) {
            if (ap64) {
                const double2 lo = *reinterpret_cast<const double2*>(ap64 + k);
                const double2 hi = *reinterpret_cast<const double2*>(ap64 + k + 2);
                a4 = make_float4((float)lo.x, (float)lo.y, (float)hi.x, (float)hi.y);
            } else if constexpr (COH) {
                // aux 16 = sc1: a device-scope load
                // (the whole vector is reinterpreted: a bit cast of one element of it loses the others)
                const f32x4g v = __builtin_bit_cast(
                    f32x4g, __builtin_amdgcn_raw_buffer_load_b128(rs, ((aok ? arow : 0) * ldin + k) * 4, 0, 16));
                a4 = make_float4(v[0], v[1], v[2], v[3]);
            } else {
                a4 = *reinterpret_cast<const float4*>(ap + k);
            }
        } else if (ap64) {
            a4.x = (aok && k < K) ? (float)ap64[k] : 0.f;
            a4.y = (aok && k + 1 < K) ? (float)ap64[k + 1] : 0.f;
            a4.z = (aok && k + 2 < K) ? (float)ap64[k + 2] : 0.f;
            a4.w = (aok && k + 3 < K) ? (float)ap64[k + 3] : 0.f;
        } else if constexpr (COH) {
            a4.x = (aok && k < K) ? coh_ld(k) : 0.f;
            a4.y = (aok && k + 1 < K) ? coh_ld(k + 1) : 0.f;
            a4.z = (aok && k + 2 < K) ? coh_ld(k + 2) : 0.f;
            a4.w = (aok && k + 3 < K) ? coh_ld(k + 3) : 0.f;
        } else {
            a4.x = (aok && k < K) ? ap[k] : 0.f;
            a4.y = (aok && k + 1 < K) ? ap[k + 1] : 0.f;
            a4.z = (aok && k + 2 < K) ? ap[k + 2] : 0.f;
            a4.w = (aok && k + 3 < K) ? ap[k + 3] : 0.f;
        }
    };
    auto load_w = [&](int t, float4& w4) {
        const int k = 8 * t + 4 * h;
        if (vec && k + 3 < K) {
            w4 = *reinterpret_cast<const float4*>(wp + k);  // rows past N: row 0, for unstored columns
        } else {
            w4.x = (wok && k < K) ? wp[k] : 0.f;
            w4.y = (wok && k + 1 < K) ? wp[k + 1] : 0.f;
            w4.z = (wok && k + 2 < K) ? wp[k + 2] : 0.f;
            w4.w = (wok && k + 3 < K) ? wp[k + 3] : 0.f;
        }
    };
    auto mfma4 = [&](const float4& a4, const float4& w4) {
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, w4.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, w4.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, w4.z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, w4.w, acc, 0, 0, 0);
    };
    // the epilogue's operands are loaded ahead, their latency hidden behind the products:
    // lane (j, h) of wave w finishes column n0 + j of rows m0 + 8 w + 4 h + 0..3
    const int n = n0 + l32;
    const bool nok = n < N;
    const float bn = (b && nok) ? b[n] : 0.f;
    float res[4] = {0.f, 0.f, 0.f, 0.f};
    auto load_res = [&] {
        if (kind != DINO_LAYER_RESID || !nok) return;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int m = m0 + 8 * wave + 4 * h + qq;
            if (m >= M) continue;
            if (in64) res[qq] = (float)in64[(long)m * ldin + n];
            else if constexpr (COH) res[qq] = __hip_atomic_load(in + (long)m * ldin + n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else res[qq] = in[(long)m * ldin + n];
        }
    };
    constexpr int PRE = 16;  // chunks per wave with all loads issued before the products
    if (nchunk <= 4 * PRE) {
        // wave w takes a contiguous quarter of K: its lanes read whole cache lines of their rows
        const int per = (nchunk + 3) / 4;
        float4 a4[PRE], w4[PRE];
#pragma unroll
        for (int u = 0; u < PRE; ++u) {
            const int t = wave * per + u;
            if (u < per && t < nchunk) load_w(t, w4[u]);
        }
        wait();
#pragma unroll
        for (int u = 0; u < PRE; ++u) {
            const int t = wave * per + u;
            if (u < per && t < nchunk) load_a(t, a4[u]);
        }
        load_res();
#pragma unroll
        for (int u = 0; u < PRE; ++u)
            if (u < per && wave * per + u < nchunk) mfma4(a4[u], w4[u]);
    } else {
        wait();
        load_res();
        for (int t = wave; t < nchunk; t += 4) {
            float4 a4, w4;
            load_w(t, w4);
            load_a(t, a4);
            mfma4(a4, w4);
        }
    }
    // split-K partial sums meet in LDS; wave w finishes registers 4w..4w+3 of the tile
    // (rows m0 + 8w + 4h + 0..3), so the epilogue runs on all four waves
#pragma unroll
    for (int q = 0; q < 16; ++q) red[wave][lane][q] = acc[q];
    __syncthreads();
    if (!nok) return;
    const float nan = __builtin_nanf("");
    const bool bad = poison != 0;
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
        const int q = 4 * wave + qq;
        const int m = m0 + 8 * wave + 4 * h + qq;
        if (m >= M) continue;
        const float z = bad ? nan : red[0][lane][q] + red[1][lane][q] + red[2][lane][q] + red[3][lane][q] + bn;
        float o;
        if (kind == DINO_LAYER_LINEAR) {
            o = z;
        } else {
            o = gelu_t<float>(z);
            if (kind == DINO_LAYER_RESID) o += res[qq];
            if (dprime) dprime[(long)m * ldd + n] = gelu_prime_t<float>(z);
        }
        if (coh_out) __hip_atomic_store(out + (long)m * ldout + n, o, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else out[(long)m * ldout + n] = o;
    }
}

__global__ __launch_bounds__(256) void fwd_mfma_kernel(int M, int K, int N, const float* __restrict__ in, int ldin,
                                                       const double* __restrict__ in64,
                                                       const float* __restrict__ W, const float* __restrict__ b,
                                                       int kind, float* __restrict__ out, int ldout,
                                                       float* __restrict__ dprime, int ldd, const int* m_dev,
                                                       int xcd_map) {
    // in64 (first layer): the FP64 states, rounded to FP32 as they are loaded
    __shared__ float red[4][64][17];
    // 1-D grid of nx * ny tiles. Blocks are dispatched round-robin over the 8 XCDs; when
    // ny is a multiple of 8, every tile of row block y goes to XCD y % 8, so that the next
    // layer's blocks of that row block read activations written through the same L2.
    const int nx = (N + 31) / 32, ny = (M + 31) / 32;
    int tx, ty;
    if (xcd_map && (ny & 7) == 0) {
        const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
        ty = xcd + 8 * (slot / nx);
        tx = slot % nx;
    } else {
        tx = blockIdx.x % nx;
        ty = blockIdx.x / nx;
    }
    const int m0 = ty * 32, n0 = tx * 32;
    if (m_dev && m0 >= *m_dev) return;  // no input rows in this tile (uniform over the block)
    const int no_poison = 0;
    fwd_tile<false>(M, K, N, in, ldin, in64, W, b, kind, out, ldout, dprime, ldd, m0, n0, red, [] {}, false,
                    no_poison);
}

// The whole FP32 forward in one launch. Block (ty, tx) owns output tile (ty, tx) of every
// layer (tiles past a layer's width idle). Layer l of row block ty starts once every tile
// of row block ty of layer l - 1 is written; counter (ty, l - 1) counts them. The hand-off
// needs no cache write-back or invalidation: the hidden activations are written with
// device-scope (sc1) stores, each wave waits for its stores to complete before thread 0
// bumps the counter (an atomic, coherent across the XCDs), and the consumers read the
// activations with device-scope loads after thread 0 has seen the count. The weight loads
// of a tile are issued before its wait. Row blocks run through the layers independently:
// no grid-wide barrier. Every block of the grid must be resident at once (the host checks
// the occupancy before choosing this kernel). A poll that gives up after FWD_SPIN_LIMIT
// rounds poisons the block's later outputs with NaN instead of waiting on, so the launch
// always ends. The last block of a row block to finish clears its counters, which are
// therefore zero between launches.
constexpr int FWD_MAXL = 16;
constexpr uint32_t FWD_SPIN_LIMIT = 1u << 20;
struct FwdLayer32 {
    const float* W;
    const float* b;
    float* out;
    float* dprime;
    int K, N, ldout, kind;
};
struct FwdChainArgs {
    int M, L, nxmax, ldin0, ldd;
    const float* in32;    // the first layer's input rows (FP32), or
    const double* in64;   // the FP64 states, rounded to FP32 as they are loaded
    uint32_t* sync;       // ceil(M / 32) x (L + 1) counters
    FwdLayer32 layer[FWD_MAXL];
};

__global__ __launch_bounds__(256) void fwd_chain32_kernel(FwdChainArgs a) {
    __shared__ float red[4][64][17];
    __shared__ int poisoned;
    const int tid = threadIdx.x;
    const int nx = a.nxmax, ny = (a.M + 31) / 32;
    int tx, ty;
    if ((ny & 7) == 0) {  // every tile of row block y on XCD y % 8, as in fwd_mfma_kernel
        const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
        ty = xcd + 8 * (slot / nx);
        tx = slot % nx;
    } else {
        tx = blockIdx.x % nx;
        ty = blockIdx.x / nx;
    }
    uint32_t* cnt = a.sync + (long)ty * (a.L + 1);
    if (tid == 0) poisoned = 0;
    __syncthreads();
    for (int l = 0; l < a.L; ++l) {
        const FwdLayer32& ly = a.layer[l];
        const bool last = l + 1 == a.L;
        // layer l of row block ty waits for every tile of layer l - 1 of that row block
        auto wait = [&] {
            if (l == 0) return;
            if (tid == 0) {
                const uint32_t want = (uint32_t)((a.layer[l - 1].N + 31) / 32);
                uint32_t spins = 0;
                while (__hip_atomic_load(cnt + l - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins >= FWD_SPIN_LIMIT) {
                        poisoned = 1;
                        break;
                    }
                }
            }
            __syncthreads();
        };
        if (tx < (ly.N + 31) / 32) {
            if (l == 0)
                fwd_tile<false>(a.M, ly.K, ly.N, a.in32, a.ldin0, a.in64, ly.W, ly.b, ly.kind, ly.out, ly.ldout,
                                ly.dprime, a.ldd, ty * 32, tx * 32, red, wait, !last, poisoned);
            else
                fwd_tile<true>(a.M, ly.K, ly.N, a.layer[l - 1].out, a.layer[l - 1].ldout, nullptr, ly.W, ly.b,
                               ly.kind, ly.out, ly.ldout, ly.dprime, a.ldd, ty * 32, tx * 32, red, wait, !last,
                               poisoned);
            if (!last) {
                // the wave's device-scope stores are complete before the count moves
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                __syncthreads();
                if (tid == 0) __hip_atomic_fetch_add(cnt + l, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    if (tid == 0) {
        // every block of this row block has passed its last poll once all nx have arrived
        const uint32_t prev = __hip_atomic_fetch_add(cnt + a.L, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (prev + 1 == (uint32_t)nx)
            for (int l = 0; l <= a.L; ++l) __hip_atomic_store(cnt + l, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <typename T>
static void fwd_layer(int M, int K, int N, const T* in, int ldin, const T* W, const T* b, int kind, T* out,
                      int ldout, T* dprime, int ldd, hipStream_t st, const int* m_dev = nullptr) {
    auto blocks = [&](int bm, int bn) { return (long)((M + bm - 1) / bm) * ((N + bn - 1) / bn); };
    // tile 0: 16 x 16, 1: 32 x 32, 2: 64 x 64 outputs per block; a tuning entry for the
    // shape decides, else the largest tile that still gives 1024 blocks
    int tile = tuned_choice(TUNE_FWD64, M, K, N);
    if (tile < 0 || tile > 2) tile = blocks(64, 64) >= 1024 ? 2 : (blocks(32, 32) >= 1024 ? 1 : 0);
    if (tile == 2)
        hipLaunchKernelGGL((fwd_layer_kernel<T, 4, 4>), dim3((N + 63) / 64, (M + 63) / 64), dim3(256), 0, st, M, K, N,
                           in, ldin, W, b, kind, out, ldout, dprime, ldd, m_dev);
    else if (tile == 1)
        hipLaunchKernelGGL((fwd_layer_kernel<T, 2, 2>), dim3((N + 31) / 32, (M + 31) / 32), dim3(256), 0, st, M, K, N,
                           in, ldin, W, b, kind, out, ldout, dprime, ldd, m_dev);
    else
        hipLaunchKernelGGL((fwd_layer_kernel<T, 1, 1>), dim3((N + 15) / 16, (M + 15) / 16), dim3(256), 0, st, M, K, N,
                           in, ldin, W, b, kind, out, ldout, dprime, ldd, m_dev);
}

// Observation-space Gram matrix I + B B^T of the FP64 path (lower triangle, d_y x d_y)
// from B = Gamma^-1/2 J (d_y x r per chain); one block per chain.
__global__ __launch_bounds__(256) void gram_f64_kernel(int dy, int r, const double* __restrict__ B, double* A,
                                                       long strideA, const int32_t* slot, int slot_xor,
                                                       long slot_stride) {
    const int c = blockIdx.x;
    const double* Bc = B + (long)c * dy * r;
    double* Ac = A + (long)c * strideA + (slot ? (long)(slot[c] ^ slot_xor) * slot_stride : 0);
    const int npairs = dy * (dy + 1) / 2;
    for (int e = threadIdx.x; e < npairs; e += 256) {
        int i = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
        while ((i + 1) * (i + 2) / 2 <= e) ++i;
        while (i * (i + 1) / 2 > e) --i;
        const int k = e - i * (i + 1) / 2;
        double acc = (i == k) ? 1.0 : 0.0;
        for (int j = 0; j < r; ++j) acc += Bc[(long)i * r + j] * Bc[(long)k * r + j];
        Ac[(long)i * dy + k] = acc;
    }
}

// H = B^T B (full r x r, FP64 products of the stored B values) per chain.
template <typename TB>
__global__ void btb_kernel(int dy, int r, int ldb, const TB* __restrict__ B, double* __restrict__ H) {
    const int c = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= r * r) return;
    const int j = e / r, k = e % r;
    const TB* Bc = B + (long)c * dy * ldb;
    double acc = 0.0;
    for (int i = 0; i < dy; ++i) acc += to_d(Bc[(long)i * ldb + j]) * to_d(Bc[(long)i * ldb + k]);
    H[(long)c * r * r + e] = acc;
}

void launch_gram_f64(dino_problem* p, int n, const double* B, double* A, long strideA, const int32_t* slot,
                     int slot_xor, long slot_stride, hipStream_t st) {
    hipLaunchKernelGGL(gram_f64_kernel, dim3(n), dim3(256), 0, st, p->d_y, p->r, B, A, strideA, slot, slot_xor,
                       slot_stride);
    DINO_HIP(hipGetLastError());
}

void launch_btb(dino_problem* p, int n, double* H, hipStream_t st) {
    const dim3 grid((p->r * p->r + 255) / 256, n);
    if (p->desc.precision == DINO_PREC_F64)
        hipLaunchKernelGGL(btb_kernel<double>, grid, dim3(256), 0, st, p->d_y, p->r, p->r, (const double*)p->Bj, H);
    else
        hipLaunchKernelGGL(btb_kernel<__hip_bfloat16>, grid, dim3(256), 0, st, p->d_y, p->r, (p->r + 31) / 32 * 32,
                           (const __hip_bfloat16*)p->B16, H);
    DINO_HIP(hipGetLastError());
}

void launch_forward(dino_problem* p, int n, const double* x, double* f_out, hipStream_t st) {
    const dino_ctx* ctx = p->ctx;
    const int L = (int)ctx->layers.size();
    const double* in = x;
    int ldin = p->r;
    int act = 0;
    for (int l = 0; l < L; ++l) {
        const Layer& ly = ctx->layers[l];
        const bool last = (l == L - 1);
        double* out;
        int ldout;
        if (last) {
            // only the observed outputs are needed
            out = f_out;
            ldout = p->d_y;
        } else {
            out = (l % 2 == 0) ? p->h0 : p->h1;
            ldout = p->wmax;
        }
        const int N = last ? p->d_y : ly.fan_out;
        double* dp = nullptr;
        if (ly.kind != DINO_LAYER_LINEAR) dp = p->dprime + (long)act * p->C * p->wmax;
        fwd_layer<double>(n, ly.fan_in, N, in, ldin, ly.W64, ly.b64, ly.kind, out, ldout, dp, p->wmax, st);
        if (ly.kind != DINO_LAYER_LINEAR) ++act;
        in = out;
        ldin = ldout;
    }
    DINO_HIP(hipGetLastError());
}

// Block order of an FP32 forward layer: 1 groups the tiles of a 32-row block on one XCD
// (when the row blocks divide by 8), 0 takes tiles in plain row-major order; a tuning
// entry for the shape decides, else the XCD grouping.
static int fwd32_xcd_map(int M, int K, int N) {
    const int t = tuned_choice(TUNE_FWD32, M, K, N);
    return t == 0 ? 0 : 1;
}

// Blocks of fwd_chain32_kernel that one device holds at once (0 if the query fails).
int fwd_chain_capacity(int device) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fwd_chain32_kernel, 256, 0) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    return per_cu * cus;
}

// Blocks of the one-launch forward of n rows (widest layer's tiles x row blocks).
static long fwd_chain_blocks(const dino_problem* p, int n) {
    const auto& ls = p->ctx->layers;
    int nx = 0;
    for (size_t l = 0; l < ls.size(); ++l) {
        const int N = (l + 1 == ls.size()) ? p->d_y : ls[l].fan_out;
        nx = std::max(nx, (N + 31) / 32);
    }
    return (long)nx * ((n + 31) / 32);
}

// The forward in one launch (fwd_chain32_kernel) where the tuning entry (chains, layers,
// widest layer) asks for it and its blocks are all resident at once; one launch per layer
// otherwise.
bool fwd_chain_usable(const dino_problem* p, int n) {
    if (!p->fsync || (int)p->ctx->layers.size() > FWD_MAXL) return false;
    if (fwd_chain_blocks(p, n) > p->fwd_chain_cap) return false;
    return tuned_choice(TUNE_FWDCHAIN, n, (int)p->ctx->layers.size(), p->wmax) == 1;
}

// FP32 forward of the mixed-precision path: gelu'(z) into d32 (row length ldd32).
void launch_forward32(dino_problem* p, int n, const float* xf, const double* x64, float* f_out, hipStream_t st) {
    const dino_ctx* ctx = p->ctx;
    const int L = (int)ctx->layers.size();
    if (fwd_chain_usable(p, n)) {
        FwdChainArgs a{};
        a.M = n;
        a.L = L;
        a.ldin0 = p->r;
        a.ldd = p->ldd32;
        a.in32 = x64 ? nullptr : xf;
        a.in64 = x64;
        a.sync = p->fsync;
        int act = 0, nx = 0;
        for (int l = 0; l < L; ++l) {
            const Layer& ly = ctx->layers[l];
            const bool last = (l == L - 1);
            FwdLayer32& d = a.layer[l];
            d.W = ly.W32;
            d.b = ly.b32;
            d.out = last ? f_out : ((l % 2 == 0) ? p->h0f : p->h1f);
            d.ldout = last ? p->d_y : p->wmax;
            d.N = last ? p->d_y : ly.fan_out;
            d.K = ly.fan_in;
            d.kind = ly.kind;
            d.dprime = nullptr;
            if (ly.kind != DINO_LAYER_LINEAR) d.dprime = p->d32 + (long)act++ * p->C * p->ldd32;
            nx = std::max(nx, (d.N + 31) / 32);
        }
        a.nxmax = nx;
        hipLaunchKernelGGL(fwd_chain32_kernel, dim3(nx * ((n + 31) / 32)), dim3(256), 0, st, a);
        DINO_HIP(hipGetLastError());
        return;
    }
    const float* in = x64 ? nullptr : xf;
    int ldin = p->r;
    int act = 0;
    for (int l = 0; l < L; ++l) {
        const Layer& ly = ctx->layers[l];
        const bool last = (l == L - 1);
        float* out = last ? f_out : ((l % 2 == 0) ? p->h0f : p->h1f);
        const int ldout = last ? p->d_y : p->wmax;
        const int N = last ? p->d_y : ly.fan_out;
        float* dp = nullptr;
        if (ly.kind != DINO_LAYER_LINEAR) dp = p->d32 + (long)act * p->C * p->ldd32;
        // the first layer reads the FP64 states (x64) when given, else the FP32 copy xf
        hipLaunchKernelGGL(fwd_mfma_kernel, dim3(((N + 31) / 32) * ((n + 31) / 32)), dim3(256), 0, st, n, ly.fan_in, N,
                           in, ldin, l == 0 ? x64 : nullptr, ly.W32, ly.b32, ly.kind, out, ldout, dp, p->ldd32,
                           (const int*)nullptr, fwd32_xcd_map(n, ly.fan_in, N));
        if (ly.kind != DINO_LAYER_LINEAR) ++act;
        in = out;
        ldin = ldout;
    }
    DINO_HIP(hipGetLastError());
}

// Forward of the true-model stand-in (delayed acceptance, second stage) on rows of zin
// (n x r_T FP64), in the problem's forward precision: FP64 layers on the FP64 path,
// FP32 MFMA layers (the first rounding zin as it loads) on the mixed path. Outputs the
// first d_y true outputs into p->fT64 or p->fT32 (n x d_y). m_dev: optional device count
// of the rows that hold input (the compacted first-stage passes).
void launch_true_forward(dino_problem* p, int n, const double* zin, const int* m_dev, hipStream_t st) {
    const auto& TL = p->ctx->true_layers;
    const int L = (int)TL.size();
    const int dy = p->d_y, wT = p->ctx->true_max_width;
    if (p->desc.precision == DINO_PREC_F64) {
        const double* in = zin;
        int ldin = p->rT;
        for (int l = 0; l < L; ++l) {
            const Layer& ly = TL[l];
            const bool last = (l == L - 1);
            double* out = last ? p->fT64 : ((l % 2 == 0) ? p->th0 : p->th1);
            const int ldout = last ? dy : wT;
            const int N = last ? dy : ly.fan_out;
            fwd_layer<double>(n, ly.fan_in, N, in, ldin, ly.W64, ly.b64, ly.kind, out, ldout, nullptr, 0, st, m_dev);
            in = out;
            ldin = ldout;
        }
    } else {
        const float* in = nullptr;
        int ldin = p->rT;
        for (int l = 0; l < L; ++l) {
            const Layer& ly = TL[l];
            const bool last = (l == L - 1);
            float* out = last ? p->fT32 : ((l % 2 == 0) ? p->th0f : p->th1f);
            const int ldout = last ? dy : wT;
            const int N = last ? dy : ly.fan_out;
            hipLaunchKernelGGL(fwd_mfma_kernel, dim3(((N + 31) / 32) * ((n + 31) / 32)), dim3(256), 0, st, n, ly.fan_in,
                               N, in, ldin, l == 0 ? zin : nullptr, ly.W32, ly.b32, ly.kind, out, ldout,
                               (float*)nullptr, 0, m_dev, fwd32_xcd_map(n, ly.fan_in, N));
            in = out;
            ldin = ldout;
        }
    }
    DINO_HIP(hipGetLastError());
}

void launch_gemm_nt64(int M, int K, int N, const double* A, int lda, const double* B, double* C, int ldc,
                      const int* m_dev, hipStream_t st) {
    fwd_layer<double>(M, K, N, A, lda, B, nullptr, DINO_LAYER_LINEAR, C, ldc, nullptr, 0, st, m_dev);
    DINO_HIP(hipGetLastError());
}

void launch_gemm_nt32(int M, int K, int N, const float* A, int lda, const float* B, float* C, int ldc,
                      const int* m_dev, hipStream_t st) {
    hipLaunchKernelGGL(fwd_mfma_kernel, dim3(((N + 31) / 32) * ((M + 31) / 32)), dim3(256), 0, st, M, K, N, A, lda,
                       (const double*)nullptr, B, (const float*)nullptr, (int)DINO_LAYER_LINEAR, C, ldc,
                       (float*)nullptr, 0, m_dev, fwd32_xcd_map(M, K, N));
    DINO_HIP(hipGetLastError());
}

void launch_reverse_jacobian(dino_problem* p, int n, double* B_out, hipStream_t st) {
    const dino_ctx* ctx = p->ctx;
    const int L = (int)ctx->layers.size();
    const int dy = p->d_y;
    const Layer& outl = ctx->layers[L - 1];
    double* cur = p->lam0;
    double* nxt = p->lam1;
    const int ld = p->wmax;
    {
        const long total = (long)n * dy * outl.fan_in;
        const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
        hipLaunchKernelGGL(rev_init_kernel<double>, dim3(blocks), dim3(256), 0, st, n, dy, outl.fan_in, outl.W64,
                           p->winv, p->meta.row, cur, ld);
    }
    int act = p->n_act;
    const int M = n * dy;
    for (int l = L - 2; l >= 0; --l) {
        const Layer& ly = ctx->layers[l];
        const double* d = nullptr;
        if (ly.kind != DINO_LAYER_LINEAR) {
            --act;
            d = p->dprime + (long)act * p->C * p->wmax;
        }
        const bool first = (l == 0);
        double* out = first ? B_out : nxt;
        const int ldo = first ? p->r : ld;
        auto kern = (M + 63) / 64 > (int)GRID_Y_MAX ? rev_layer_kernel<double, true> : rev_layer_kernel<double, false>;
        hipLaunchKernelGGL(kern, grid2(M, ly.fan_in), dim3(256), 0, st, M, ly.fan_out,
                           ly.fan_in, dy, cur, ld, d, p->wmax, ly.W64, ly.kind == DINO_LAYER_RESID ? 1 : 0, out,
                           ldo);
        if (!first) std::swap(cur, nxt);
    }
    DINO_HIP(hipGetLastError());
}

void launch_misfit_grad(dino_problem* p, int n, const double* f, const double* B, double* phi, double* g,
                        hipStream_t st) {
    hipLaunchKernelGGL(misfit_grad_kernel, dim3(n), dim3(256), 0, st, n, p->d_y, p->r, f, p->y, p->winv,
                       p->meta.row, B, phi, g);
    DINO_HIP(hipGetLastError());
}

void launch_gn_hessian_slot(dino_problem* p, int n, const double* B, double* A, long strideA,
                            const int32_t* slot, int slot_xor, long slot_stride, int add_identity, int full,
                            hipStream_t st) {
    const int t = (p->r + 31) / 32;
    auto kern = n > (int)GRID_Y_MAX ? gn_hessian_kernel<true> : gn_hessian_kernel<false>;
    hipLaunchKernelGGL(kern, dim3(t, t, grid_y(n)), dim3(256), 0, st, n, p->d_y, p->r, B, A, strideA, slot,
                       slot_xor, slot_stride, add_identity, full);
    DINO_HIP(hipGetLastError());
}

}  // namespace dino
