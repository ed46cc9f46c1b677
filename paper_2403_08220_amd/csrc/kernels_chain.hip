// Per-chain FP64 kernels of the reduced mMALA transition:
//  * Cholesky factor of I + H (replaces the eigendecomposition of Sec. 5.2),
//  * reduced proposal (splitting proposition of Sec. 5.3, item 2, eq. reduced_space_sampling),
//  * reduced RN derivative and first-stage ratio (Sec. 5.4, eq. da_dino_trr_1),
//  * MH decision (Alg. 1: reject iff alpha < xi_1) and state swap,
//  * pCN move of the complement (splitting proposition of Sec. 5.3, item 1), trace rows, draws.
#include "dino_internal.hpp"
#include "chol_wave.hpp"

namespace dino {

constexpr int TPB = 256;      // threads per block of the per-chain kernels
constexpr int MAXR = 512;     // largest reduced dimension of the per-chain kernels
constexpr int SB = 32;        // block size of the triangular solves

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Value of lane `lane` (wave-uniform) of a double, through two v_readlane (a scalar
// broadcast, far shorter latency than a cross-lane permute).
__device__ __forceinline__ double lane_bcast(double v, int lane) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sums over the block of four values per thread at once; red must hold 4 * TPB/64
// doubles.
__device__ __forceinline__ void block_sum4(double (&v)[4], double* red) {
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = wave_sum(v[q]);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q) red[4 * wave + q] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < TPB / 64; ++k) t += red[4 * k + q];
        v[q] = t;
    }
}

// Sum over the block of one value per thread; red must hold TPB/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < TPB / 64; ++k) t += red[k];
    return t;
}

// Backward substitution L^T x = b. Blocks from the bottom: rows of the block subtract
// the solved part below through column reads (32 consecutive columns per row), then
// lanes 0..SB-1 of wave 0 finish the block's transposed triangle. In that serial part
// lane l keeps the numerator a_l of x_l; the triangle entries are pre-scaled,
// L_jl / L_jj (zero unless l < j), so that step j is one broadcast of a_j and one FMA
// per lane, and x_l = a_l / L_ll at the end.
__device__ __forceinline__ void lt_solve(const double* __restrict__ L, const double* invd, int r, const double* b, double* x,
                         double* part) {
    const int tid = threadIdx.x;
    const int nblk = (r + SB - 1) / SB;
    for (int bi = nblk - 1; bi >= 0; --bi) {
        const int b0 = bi * SB;
        const int nb = min(SB, r - b0);
        // wave 0 issues the loads of the block's triangle before the partial sums
        double col[SB];
        if (tid < 64) {
            const int lane = tid;
#pragma unroll
            for (int jj = 0; jj < SB; ++jj)
                col[jj] = (lane < nb && jj > lane && jj < nb) ? L[(long)(b0 + jj) * r + b0 + lane] : 0.0;
        }
        {
            const int il = tid & 31, grp = tid >> 5;  // 32 columns x 8 row groups
            double acc = 0.0;
            constexpr int PB = 8;  // loads issued before their products
            if (il < nb)
                for (int j0 = b0 + nb + grp; j0 < r; j0 += 8 * PB) {
                    double lv[PB];
#pragma unroll
                    for (int u = 0; u < PB; ++u) lv[u] = (j0 + 8 * u < r) ? L[(long)(j0 + 8 * u) * r + b0 + il] : 0.0;
#pragma unroll
                    for (int u = 0; u < PB; ++u)
                        if (j0 + 8 * u < r) acc += lv[u] * x[j0 + 8 * u];
                }
            part[grp * SB + il] = acc;
        }
        __syncthreads();
        if (tid < 64) {
            const int lane = tid;
            double a = 0.0;
            if (lane < nb) {
                double s = 0.0;
#pragma unroll
                for (int g = 0; g < 8; ++g) s += part[g * SB + lane];
                a = b[b0 + lane] - s;
            }
            // entries past the block are zero: the clamped index only keeps the factor finite
#pragma unroll
            for (int jj = 0; jj < SB; ++jj) col[jj] *= invd[min(b0 + jj, r - 1)];
#pragma unroll
            for (int jj = SB - 1; jj >= 0; --jj) a -= col[jj] * lane_bcast(a, jj);
            if (lane < nb) x[b0 + lane] = a * invd[b0 + lane];
        }
        __syncthreads();
    }
}

// 1 / L_jj for j < r into LDS (the solves multiply instead of dividing).
__device__ __forceinline__ void load_inv_diag(const double* __restrict__ L, int r, double* invd, bool sync = true) {
    for (int j = threadIdx.x; j < r; j += TPB) invd[j] = 1.0 / L[(long)j * r + j];
    if (sync) __syncthreads();
}

// out1_j = sum_{i >= j} L[i][j] v1_i (L^T v1) and, if v2, out2 = L^T v2, in one pass
// over L. Waves take rows i = wave (mod 4); lanes read 64 consecutive columns of a row;
// partial sums are reduced through part (4 r doubles per product).
__device__ __forceinline__ void lt_matvec2(const double* __restrict__ L, int r, const double* v1, double* out1, const double* v2,
                           double* out2, double* part) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int jb = 0; jb < r; jb += 64) {
        const int j = jb + lane;
        double a1 = 0.0, a2 = 0.0;
        if (j < r) {
#pragma unroll 8
            for (int i = jb + ((wave - jb) & 3); i < r; i += 4) {
                if (i >= j) {
                    const double lij = L[(long)i * r + j];
                    a1 += lij * v1[i];
                    if (v2) a2 += lij * v2[i];
                }
            }
            part[wave * r + j] = a1;
            if (v2) part[(4 + wave) * r + j] = a2;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < r; j += TPB) {
        out1[j] = part[j] + part[r + j] + part[2 * r + j] + part[3 * r + j];
        if (v2) out2[j] = part[4 * r + j] + part[5 * r + j] + part[6 * r + j] + part[7 * r + j];
    }
    __syncthreads();
}

// Forward substitution L w = b (L lower, non-singular). Block rows of SB: the rows of
// a block first subtract the already solved part (8 threads per row), then lanes
// 0..SB-1 of wave 0 finish the block's triangle with register broadcasts: lane l keeps
// the numerator a_l of w_l, the triangle entries are pre-scaled, L_lj / L_jj (zero
// unless j < l), so step j is one broadcast of a_j and one FMA per lane, and
// w_l = a_l / L_ll at the end.
__device__ __forceinline__ void l_solve(const double* __restrict__ L, const double* invd, int r, const double* b, double* w,
                        double* acc_s) {
    const int tid = threadIdx.x;
    for (int b0 = 0; b0 < r; b0 += SB) {
        const int nb = min(SB, r - b0);
        // wave 0 issues the loads of the block's triangle before the partial sums, so that
        // both wait for memory once
        double row[SB];
        if (tid < 64) {
            const int lane = tid;
#pragma unroll
            for (int jj = 0; jj < SB; ++jj)
                row[jj] = (lane < nb && jj < lane) ? L[(long)(b0 + lane) * r + b0 + jj] : 0.0;
        }
        {
            const int il = tid >> 3, sub = tid & 7;  // 32 rows x 8 threads
            const int i = b0 + il;
            double acc = 0.0;
            // j + 3 < b0 whenever j < b0 (b0 is a multiple of 32); the loads of PB
            // chunks are issued before their products
            constexpr int PB = 4;
            if (il < nb)
                for (int j0 = 4 * sub; j0 < b0; j0 += 32 * PB) {
                    double lv[PB][4];
#pragma unroll
                    for (int u = 0; u < PB; ++u)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            lv[u][q] = (j0 + 32 * u < b0) ? L[(long)i * r + j0 + 32 * u + q] : 0.0;
#pragma unroll
                    for (int u = 0; u < PB; ++u)
                        if (j0 + 32 * u < b0)
#pragma unroll
                            for (int q = 0; q < 4; ++q) acc += lv[u][q] * w[j0 + 32 * u + q];
                }
#pragma unroll
            for (int o = 4; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
            if (il < nb && sub == 0) acc_s[il] = b[i] - acc;
        }
        __syncthreads();
        if (tid < 64) {
            const int lane = tid;
            double a = lane < nb ? acc_s[lane] : 0.0;
            // entries past the block are zero: the clamped index only keeps the factor finite
#pragma unroll
            for (int jj = 0; jj < SB; ++jj) row[jj] *= invd[min(b0 + jj, r - 1)];
#pragma unroll
            for (int jj = 0; jj < SB; ++jj) a -= row[jj] * lane_bcast(a, jj);
            if (lane < nb) w[b0 + lane] = a * invd[b0 + lane];
        }
        __syncthreads();
    }
}

// out = L^T v (L lower, row stride r): waves take rows i = wave (mod 4), lanes 64
// consecutive columns j <= i, with the loads of PB rows issued before their products;
// the four waves' partial sums meet in part (4 x 64 doubles) and are added in wave
// order.
__device__ __forceinline__ void lt_matvec(const double* __restrict__ L, int r, const double* v, double* out,
                                          double* part) {
    static_assert(TPB == 256, "four waves");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int PB = 16;
    for (int jb = 0; jb < r; jb += 64) {
        const int j = jb + lane;
        double a = 0.0;
        if (j < r) {
            for (int i0 = jb + ((wave - jb) & 3); i0 < r; i0 += 4 * PB) {
                double lv[PB];
#pragma unroll
                for (int u = 0; u < PB; ++u) {
                    const int i = i0 + 4 * u;
                    lv[u] = (i < r && i >= j) ? L[(long)i * r + j] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < PB; ++u) {
                    const int i = i0 + 4 * u;
                    if (i < r && i >= j) a += lv[u] * v[i];
                }
            }
        }
        part[wave * 64 + lane] = a;
        __syncthreads();
        if (wave == 0 && j < r) out[j] = part[lane] + part[64 + lane] + part[128 + lane] + part[192 + lane];
        __syncthreads();
    }
}

// Forward substitution for two right-hand sides at once (L w1 = b1, L w2 = b2): one
// pass over L and one serial sweep for both (as l_solve); acc_s must hold 2 SB doubles.
__device__ __forceinline__ void l_solve2(const double* __restrict__ L, const double* invd, int r, const double* b1,
                                         double* w1, const double* b2, double* w2, double* acc_s) {
    const int tid = threadIdx.x;
    for (int b0 = 0; b0 < r; b0 += SB) {
        const int nb = min(SB, r - b0);
        double row[SB];
        if (tid < 64) {
            const int lane = tid;
#pragma unroll
            for (int jj = 0; jj < SB; ++jj)
                row[jj] = (lane < nb && jj < lane) ? L[(long)(b0 + lane) * r + b0 + jj] : 0.0;
        }
        {
            const int il = tid >> 3, sub = tid & 7;  // 32 rows x 8 threads
            const int i = b0 + il;
            double c1 = 0.0, c2 = 0.0;
            // j + 3 < b0 whenever j < b0 (b0 is a multiple of 32); the loads of PB
            // chunks are issued before their products
            constexpr int PB = 4;
            if (il < nb)
                for (int j0 = 4 * sub; j0 < b0; j0 += 32 * PB) {
                    double lv[PB][4];
#pragma unroll
                    for (int u = 0; u < PB; ++u)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            lv[u][q] = (j0 + 32 * u < b0) ? L[(long)i * r + j0 + 32 * u + q] : 0.0;
#pragma unroll
                    for (int u = 0; u < PB; ++u)
                        if (j0 + 32 * u < b0)
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                c1 += lv[u][q] * w1[j0 + 32 * u + q];
                                c2 += lv[u][q] * w2[j0 + 32 * u + q];
                            }
                }
#pragma unroll
            for (int o = 4; o > 0; o >>= 1) {
                c1 += __shfl_xor(c1, o);
                c2 += __shfl_xor(c2, o);
            }
            if (il < nb && sub == 0) {
                acc_s[il] = b1[i] - c1;
                acc_s[SB + il] = b2[i] - c2;
            }
        }
        __syncthreads();
        if (tid < 64) {
            const int lane = tid;
            double a1 = lane < nb ? acc_s[lane] : 0.0;
            double a2 = lane < nb ? acc_s[SB + lane] : 0.0;
            // entries past the block are zero: the clamped index only keeps the factor finite
#pragma unroll
            for (int jj = 0; jj < SB; ++jj) row[jj] *= invd[min(b0 + jj, r - 1)];
#pragma unroll
            for (int jj = 0; jj < SB; ++jj) {
                const double u1 = lane_bcast(a1, jj), u2 = lane_bcast(a2, jj);
                a1 -= row[jj] * u1;
                a2 -= row[jj] * u2;
            }
            if (lane < nb) {
                const double dl = invd[b0 + lane];
                w1[b0 + lane] = a1 * dl;
                w2[b0 + lane] = a2 * dl;
            }
        }
        __syncthreads();
    }
}

// Triangular solves with inverted diagonal blocks. The fused Gram + factor kernel also
// stores D_b = L_bb^-1 for every diagonal block b of SB rows: the strictly lower entries
// of D_b transposed in the strictly upper triangle of block (b, b) of the factor (entry
// D_b[k][m], m < k, at row b0 + m, column b0 + k); the diagonal of D_b is invd. A block of
// a solve is then w_b = D_b (b_b - the solved part), two parallel passes with the same
// thread layout (32 rows x 8 threads), instead of a serial sweep over the block's
// columns. The loads of D_b's entries go out with the partial sums' loads.

// thread (il, sub)'s entries of row il of D_b, columns 4 sub + q (zero past the diagonal)
__device__ __forceinline__ void dinv_row4(const double* __restrict__ L, int r, int b0, int nb, int il, int sub,
                                          double dv[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int m = 4 * sub + q;
        dv[q] = (il < nb && m < il) ? L[(long)(b0 + m) * r + b0 + il] : 0.0;
    }
}

// sum_m D_b[il][m] a_m over the thread's four columns (a: the block's right-hand side in
// LDS; the diagonal entry from invd), reduced over the row's 8 threads
__device__ __forceinline__ double dinv_row_dot(const double dv[4], const double* invd, int b0, int nb, int il, int sub,
                                               const double* a) {
    double s = 0.0;
    if (il < nb) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int m = 4 * sub + q;
            if (m < il) s += dv[q] * a[m];
            else if (m == il) s += invd[b0 + il] * a[m];
        }
    }
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) s += __shfl_xor(s, o);
    return s;
}

// Partial sums of rows b0 + il over the solved columns j < b0 (8 threads per row), for
// one or two right-hand sides (w2 may be null), as l_solve / l_solve2 form them.
__device__ __forceinline__ void lower_partials(const double* __restrict__ L, int r, int b0, int nb, int il, int sub,
                                               const double* w1, const double* w2, double& c1, double& c2) {
    const int i = b0 + il;
    c1 = 0.0;
    c2 = 0.0;
    constexpr int PB = 4;
    if (il < nb)
        for (int j0 = 4 * sub; j0 < b0; j0 += 32 * PB) {
            double lv[PB][4];
#pragma unroll
            for (int u = 0; u < PB; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q) lv[u][q] = (j0 + 32 * u < b0) ? L[(long)i * r + j0 + 32 * u + q] : 0.0;
#pragma unroll
            for (int u = 0; u < PB; ++u)
                if (j0 + 32 * u < b0)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        c1 += lv[u][q] * w1[j0 + 32 * u + q];
                        if (w2) c2 += lv[u][q] * w2[j0 + 32 * u + q];
                    }
        }
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) {
        c1 += __shfl_xor(c1, o);
        if (w2) c2 += __shfl_xor(c2, o);
    }
}

// L w1 = b1 and, if w2, L w2 = b2 (acc_s: 2 SB doubles).
__device__ __forceinline__ void l_solve_dinv(const double* __restrict__ L, const double* invd, int r, const double* b1,
                                             double* w1, const double* b2, double* w2, double* acc_s) {
    const int tid = threadIdx.x, il = tid >> 3, sub = tid & 7;
    for (int b0 = 0; b0 < r; b0 += SB) {
        const int nb = min(SB, r - b0), i = b0 + il;
        double dv[4];
        dinv_row4(L, r, b0, nb, il, sub, dv);
        double c1, c2;
        lower_partials(L, r, b0, nb, il, sub, w1, w2, c1, c2);
        if (il < nb && sub == 0) {
            acc_s[il] = b1[i] - c1;
            if (w2) acc_s[SB + il] = b2[i] - c2;
        }
        __syncthreads();
        const double s1 = dinv_row_dot(dv, invd, b0, nb, il, sub, acc_s);
        const double s2 = w2 ? dinv_row_dot(dv, invd, b0, nb, il, sub, acc_s + SB) : 0.0;
        if (il < nb && sub == 0) {
            w1[i] = s1;
            if (w2) w2[i] = s2;
        }
        __syncthreads();
    }
}

// L^T x = b, blocks from the bottom: x_b = D_b^T (b_b - sum over the solved rows below of
// L_jb x_j). The partial sums as lt_solve forms them (part: 8 SB doubles), the block's
// right-hand side into acc_s (SB doubles), then thread (il, sub) forms
// sum_k D_b[k][il] a_k over k = 4 sub + q (D_b[k][il] at row b0 + il, column b0 + k).
// With v2, out2 = L^T v2 rides on the same loads of L's columns (the block's own lower
// triangle loaded besides; partial sums in part2, 8 SB doubles, added in group order).
__device__ __forceinline__ void lt_solve_dinv(const double* __restrict__ L, const double* invd, int r, const double* b,
                                              double* x, double* part, double* acc_s, const double* v2 = nullptr,
                                              double* out2 = nullptr, double* part2 = nullptr) {
    const int tid = threadIdx.x;
    const int nblk = (r + SB - 1) / SB;
    for (int bi = nblk - 1; bi >= 0; --bi) {
        const int b0 = bi * SB;
        const int nb = min(SB, r - b0);
        const int il2 = tid >> 3, sub = tid & 7;
        double dv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = 4 * sub + q;
            dv[q] = (il2 < nb && k > il2 && k < nb) ? L[(long)(b0 + il2) * r + b0 + k] : 0.0;
        }
        {
            const int il = tid & 31, grp = tid >> 5;  // 32 columns x 8 row groups
            double acc = 0.0, acc2 = 0.0;
            constexpr int PB = 8;
            if (v2 && il < nb) {
                // L^T v2 over the block's own rows j >= b0 + il
                double dl[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int jj = grp + 8 * t;
                    dl[t] = (jj < nb && jj >= il) ? L[(long)(b0 + jj) * r + b0 + il] : 0.0;
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int jj = grp + 8 * t;
                    if (jj < nb && jj >= il) acc2 += dl[t] * v2[b0 + jj];
                }
            }
            if (il < nb)
                for (int j0 = b0 + nb + grp; j0 < r; j0 += 8 * PB) {
                    double lv[PB];
#pragma unroll
                    for (int u = 0; u < PB; ++u) lv[u] = (j0 + 8 * u < r) ? L[(long)(j0 + 8 * u) * r + b0 + il] : 0.0;
#pragma unroll
                    for (int u = 0; u < PB; ++u)
                        if (j0 + 8 * u < r) {
                            acc += lv[u] * x[j0 + 8 * u];
                            if (v2) acc2 += lv[u] * v2[j0 + 8 * u];
                        }
                }
            part[grp * SB + il] = acc;
            if (v2) part2[grp * SB + il] = acc2;
        }
        __syncthreads();
        if (tid < nb) {
            double s = 0.0;
#pragma unroll
            for (int g = 0; g < 8; ++g) s += part[g * SB + tid];
            acc_s[tid] = b[b0 + tid] - s;
            if (v2) {
                double s2 = 0.0;
#pragma unroll
                for (int g = 0; g < 8; ++g) s2 += part2[g * SB + tid];
                out2[b0 + tid] = s2;
            }
        }
        __syncthreads();
        double t = 0.0;
        if (il2 < nb) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 4 * sub + q;
                if (k > il2 && k < nb) t += dv[q] * acc_s[k];
                else if (k == il2) t += invd[b0 + il2] * acc_s[k];
            }
        }
#pragma unroll
        for (int o = 4; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if (il2 < nb && sub == 0) x[b0 + il2] = t;
        __syncthreads();
    }
}

// Dynamic LDS of the per-chain transition kernels: CH_NV vectors of length r, the
// triangular-solve scratch and the partial sums of the transposed products.
constexpr int CH_NV = 10;
struct ChainLds {
    double* v[CH_NV];
    double* acc;   // SB
    double* part;  // max(8 SB, 8 r)
    double* red;   // TPB / 64
};

__host__ __device__ inline size_t chain_lds_doubles(int r) {
    return (size_t)CH_NV * r + SB + (size_t)8 * max(r, SB) + TPB / 64;
}

__device__ inline ChainLds carve_chain_lds(double* base, int r) {
    ChainLds S;
#pragma unroll
    for (int k = 0; k < CH_NV; ++k) S.v[k] = base + (size_t)k * r;
    double* p = base + (size_t)CH_NV * r;
    S.acc = p;
    S.part = p + SB;
    S.red = p + SB + (size_t)8 * max(r, SB);
    return S;
}

__device__ __forceinline__ long slot_offset(const int32_t* slot, int slot_xor, long slot_stride, int c) {
    return slot ? (long)(slot[c] ^ slot_xor) * slot_stride : 0;
}

// ---------------------------------------------------------------------------------
// In-place Cholesky of A_c (r x r, lower triangle read and written): right-looking
// with 32-column panels factored in LDS; trailing update in 4x4 register blocks.
constexpr int CNB = 32;
constexpr int CLDP = CNB + 1;

__global__ __launch_bounds__(TPB) void cholesky_kernel(int r, double* A, long strideA, const int32_t* slot,
                                                       int slot_xor, long slot_stride, double* logdet,
                                                       int32_t* ok) {
    extern __shared__ double P[];  // r x CLDP
    __shared__ int fail;
    __shared__ double ld_acc;
    const int c = blockIdx.x, tid = threadIdx.x;
    double* a = A + (long)c * strideA + slot_offset(slot, slot_xor, slot_stride, c);
    if (tid == 0) {
        fail = 0;
        ld_acc = 0.0;
    }
    for (int j0 = 0; j0 < r; j0 += CNB) {
        const int jb = min(CNB, r - j0), rows = r - j0;
        for (int e = tid; e < rows * CNB; e += TPB) {
            const int i = e / CNB, jj = e % CNB;
            if (jj < jb) P[i * CLDP + jj] = a[(long)(j0 + i) * r + j0 + jj];
        }
        __syncthreads();
        // Column jj of the panel: every thread forms the pivot from the finished entry,
        // scales its rows, then threads (column kk = tid % 32, row group tid / 32) apply
        // the rank-1 update to the panel columns right of jj.
        const int kk = tid & (CNB - 1), rg = tid >> 5;
        for (int jj = 0; jj < jb; ++jj) {
            const double piv = P[jj * CLDP + jj];
            const double dgl = sqrt(piv);
            const double inv = 1.0 / dgl;
            for (int i = jj + 1 + tid; i < rows; i += TPB) P[i * CLDP + jj] *= inv;
            __syncthreads();
            if (tid == 0) {
                if (!(piv > 0.0)) fail = 1;
                else ld_acc += log(dgl);
                P[jj * CLDP + jj] = dgl;
            }
            if (kk > jj && kk < jb) {
                const double lk = P[kk * CLDP + jj];
                for (int i = kk + rg; i < rows; i += TPB / CNB) P[i * CLDP + kk] -= P[i * CLDP + jj] * lk;
            }
            __syncthreads();
        }
        for (int e = tid; e < rows * CNB; e += TPB) {
            const int i = e / CNB, jj = e % CNB;
            if (jj < jb && jj <= i) a[(long)(j0 + i) * r + j0 + jj] = P[i * CLDP + jj];
        }
        const int t0 = j0 + jb, T = r - t0;
        if (T > 0) {
            const int nbk = (T + 3) / 4;
            const int nblocks = nbk * (nbk + 1) / 2;
            for (int bidx = tid; bidx < nblocks; bidx += TPB) {
                int bi = (int)((sqrt(8.0 * (double)bidx + 1.0) - 1.0) * 0.5);
                while ((bi + 1) * (bi + 2) / 2 <= bidx) ++bi;
                while (bi * (bi + 1) / 2 > bidx) --bi;
                const int bk = bidx - bi * (bi + 1) / 2;
                double acc[4][4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int s = 0; s < 4; ++s) acc[q][s] = 0.0;
                for (int jj = 0; jj < jb; ++jj) {
                    double pi[4], pk[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int li = 4 * bi + q, lk = 4 * bk + q;
                        pi[q] = (li < T) ? P[(jb + li) * CLDP + jj] : 0.0;
                        pk[q] = (lk < T) ? P[(jb + lk) * CLDP + jj] : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int s = 0; s < 4; ++s) acc[q][s] += pi[q] * pk[s];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const int i = t0 + 4 * bi + q, k = t0 + 4 * bk + s;
                        if (i < r && k <= i) a[(long)i * r + k] -= acc[q][s];
                    }
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (logdet) logdet[c] = ld_acc;
        if (ok) ok[c] = fail ? 0 : 1;
    }
}

// In-place Cholesky of A_c (r x r, lower triangle read and written) for the largest
// orders: right-looking over 32-column panels, one 512-thread block per chain (two waves
// per SIMD). A panel is held transposed in LDS (column jj of the panel at Pt + jj LD,
// LD = r rounded up to odd, so that consecutive rows are consecutive words):
//   1. one wave factors the 32 x 32 diagonal block (lane = row, the row in registers,
//      each column's multipliers broadcast across lanes by shuffles);
//   2. the rows below are solved row-parallel, L21 = A21 L11^-T, one row per thread with
//      the row in registers;
//   3. the trailing update A22 -= L21 L21^T runs in 4 x 4 register blocks, each thread
//      loading its block of A22 before the products so that the loads' latency overlaps them.
constexpr int PTPB = 512;
constexpr int PNB = 32;

// row[lane] with a run-time lane: the diagonal entry a lane holds.
__device__ __forceinline__ double lane_diag(const double (&row)[PNB], int lane) {
    double d = 0.0;
#pragma unroll
    for (int k = 0; k < PNB; ++k)
        if (k == lane) d = row[k];
    return d;
}

__global__ __launch_bounds__(PTPB) void cholesky_panel_kernel(int r, double* A, long strideA, const int32_t* slot,
                                                             int slot_xor, long slot_stride, double* logdet,
                                                             int32_t* ok) {
    extern __shared__ double Pt[];  // PNB x LD, then the panel's reciprocal pivots
    __shared__ int fail;
    __shared__ double ld_acc;
    const int LD = r | 1;
    double* dinv = Pt + PNB * LD;
    const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* a = A + (long)c * strideA + slot_offset(slot, slot_xor, slot_stride, c);
    if (tid == 0) {
        fail = 0;
        ld_acc = 0.0;
    }
    for (int j0 = 0; j0 < r; j0 += PNB) {
        const int jb = min(PNB, r - j0), rows = r - j0;
        __syncthreads();  // the previous panel's readers are done
        // eight loads per thread in flight before their LDS stores (one load and its wait
        // per element had made the staging a chain of memory round trips)
        constexpr int PB8 = 8;
        for (int e0 = tid; e0 < rows * PNB; e0 += PB8 * PTPB) {
            double v[PB8];
#pragma unroll
            for (int u = 0; u < PB8; ++u) {
                const int e = e0 + u * PTPB, i = e >> 5, jj = e & (PNB - 1);
                v[u] = 0.0;
                if (e < rows * PNB && jj < jb && jj <= i) v[u] = a[(long)(j0 + i) * r + j0 + jj];
            }
#pragma unroll
            for (int u = 0; u < PB8; ++u) {
                const int e = e0 + u * PTPB, i = e >> 5, jj = e & (PNB - 1);
                if (e < rows * PNB && jj < jb && jj <= i) Pt[jj * LD + i] = v[u];
            }
        }
        __syncthreads();
        if (wave == 0) {
            // lane = row of the diagonal block, held in registers; column jj's pivot and
            // multipliers reach the other lanes by v_readlane (uniform lane index)
            double row[PNB];
#pragma unroll
            for (int k = 0; k < PNB; ++k) row[k] = (lane < jb && k <= lane) ? Pt[k * LD + lane] : 0.0;
            bool bad = false;
#pragma unroll
            for (int jj = 0; jj < PNB; ++jj) {
                if (jj < jb) {
                    const double piv = lane_bcast(row[jj], jj);
                    bad = bad || !(piv > 0.0);
                    const double dgl = sqrt(piv);
                    const double inv = 1.0 / dgl;
                    const double l = (lane > jj && lane < jb) ? row[jj] * inv : 0.0;
                    if (lane == jj) row[jj] = dgl;
                    if (lane > jj) row[jj] = l;
                    if (lane == 0) dinv[jj] = inv;
#pragma unroll
                    for (int k = jj + 1; k < PNB; ++k) {
                        const double lk = lane_bcast(l, k);
                        if (k <= lane) row[k] -= l * lk;  // l = 0 on lanes <= jj
                    }
                }
            }
            // log det of the block: one log per lane (its pivot), summed across the wave
            double lg = (lane < jb) ? log(lane_diag(row, lane)) : 0.0;
            for (int o = 32; o > 0; o >>= 1) lg += __shfl_xor(lg, o);
            if (lane == 0) {
                if (bad) fail = 1;
                ld_acc += lg;
            }
#pragma unroll
            for (int k = 0; k < PNB; ++k)
                if (lane < jb && k <= lane) Pt[k * LD + lane] = row[k];
        }
        __syncthreads();
        for (int i = jb + tid; i < rows; i += PTPB) {
            double x[PNB];
            if (jb == PNB) {  // full panel: one straight-line region, its LDS reads issued early
#pragma unroll
                for (int jj = 0; jj < PNB; ++jj) x[jj] = Pt[jj * LD + i];
#pragma unroll
                for (int jj = 0; jj < PNB; ++jj) {
                    double sum = x[jj];
#pragma unroll
                    for (int t = 0; t < jj; ++t) sum -= x[t] * Pt[t * LD + jj];
                    x[jj] = sum * dinv[jj];
                }
#pragma unroll
                for (int jj = 0; jj < PNB; ++jj) Pt[jj * LD + i] = x[jj];
            } else {
#pragma unroll
                for (int jj = 0; jj < PNB; ++jj) x[jj] = jj < jb ? Pt[jj * LD + i] : 0.0;
#pragma unroll
                for (int jj = 0; jj < PNB; ++jj) {
                    if (jj < jb) {
                        double sum = x[jj];
#pragma unroll
                        for (int t = 0; t < jj; ++t) sum -= x[t] * Pt[t * LD + jj];
                        x[jj] = sum * dinv[jj];
                    }
                }
#pragma unroll
                for (int jj = 0; jj < PNB; ++jj)
                    if (jj < jb) Pt[jj * LD + i] = x[jj];
            }
        }
        __syncthreads();
        for (int e = tid; e < rows * PNB; e += PTPB) {
            const int i = e >> 5, jj = e & (PNB - 1);
            if (jj < jb && jj <= i) a[(long)(j0 + i) * r + j0 + jj] = Pt[jj * LD + i];
        }
        const int T = rows - jb;
        if (T > 0) {
            const int nbk = (T + 3) / 4;
            const int nblocks = nbk * (nbk + 1) / 2;
            for (int bidx = tid; bidx < nblocks; bidx += PTPB) {
                int bi = (int)((sqrt(8.0 * (double)bidx + 1.0) - 1.0) * 0.5);
                while ((bi + 1) * (bi + 2) / 2 <= bidx) ++bi;
                while (bi * (bi + 1) / 2 > bidx) --bi;
                const int bk = bidx - bi * (bi + 1) / 2;
                const int li = jb + 4 * bi, lk = jb + 4 * bk;  // panel-local rows of the block
                double old[4][4], acc[4][4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int s2 = 0; s2 < 4; ++s2) {
                        const int i = li + q, k = lk + s2;
                        old[q][s2] = (i < rows && k <= i) ? a[(long)(j0 + i) * r + j0 + k] : 0.0;
                        acc[q][s2] = 0.0;
                    }
                for (int jj = 0; jj < jb; ++jj) {
                    double pi[4], pk[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        pi[q] = Pt[jj * LD + min(li + q, rows - 1)];
                        pk[q] = Pt[jj * LD + min(lk + q, rows - 1)];
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int s2 = 0; s2 < 4; ++s2) acc[q][s2] += pi[q] * pk[s2];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int s2 = 0; s2 < 4; ++s2) {
                        const int i = li + q, k = lk + s2;
                        if (i < rows && k <= i) a[(long)(j0 + i) * r + j0 + k] = old[q][s2] - acc[q][s2];
                    }
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        if (logdet) logdet[c] = ld_acc;
        if (ok) ok[c] = fail ? 0 : 1;
    }
}

// Register-resident Cholesky for r <= min(G MR, 32 MC), G = NT / 32: the NT threads of a
// block hold the lower triangle in a 2-D cyclic layout, thread t = 32 g + q owning rows
// i = g + G m (m < MR) and columns k = q + 32 c (c < MC). A (m, c) pair is kept only if
// it can hold a lower-triangle element (32 c <= G m + G - 1), which halves the registers.
// Column j of the Schur complement is broadcast through LDS (double buffered, one
// barrier per column); every thread then applies
//     a_ik -= a_ij a_kj / a_jj        (i, k > j)
// and the owners of column j scale it to L_ij = a_ij / sqrt(a_jj). The columns are
// walked in phases of G: within phase p the row blocks m < p and the column blocks
// c < (G p) / 32 are finished, and both bounds are compile-time constants of the
// unrolled phase, so a phase's body holds only its live updates and no skip branches.
// The pivots go to LDS; log det L = (1/2) sum_j log a_jj is reduced at the end.
template <int G>
__host__ __device__ constexpr bool chol_pair(int m, int c) { return 32 * c <= G * m + G - 1; }

template <int NT, int MR, int MC>
__global__ __launch_bounds__(NT) void cholesky_reg_kernel(int r, double* A, long strideA, const int32_t* slot,
                                                          int slot_xor, long slot_stride, double* logdet,
                                                          int32_t* ok) {
    constexpr int G = NT / 32;
    constexpr int NB = (G * MR > 32 * MC) ? G * MR : 32 * MC;
    __shared__ double colbuf[2][NB];
    __shared__ double pivs[NB];
    __shared__ double red[NT / 64];
    const int c = blockIdx.x, tid = threadIdx.x;
    const int g = tid >> 5, q = tid & 31;
    double* a = A + (long)c * strideA + slot_offset(slot, slot_xor, slot_stride, c);
    for (int e = tid; e < 2 * NB; e += NT) (&colbuf[0][0])[e] = 0.0;
    double v[MR][MC];
#pragma unroll
    for (int m = 0; m < MR; ++m) {
        const int i = g + G * m;
#pragma unroll
        for (int cc = 0; cc < MC; ++cc) {
            if (chol_pair<G>(m, cc)) {
                const int k = q + 32 * cc;
                v[m][cc] = (i < r && k <= i) ? a[i * r + k] : 0.0;
            }
        }
    }
    bool bad = false;
#pragma unroll
    for (int ph = 0; ph < MR; ++ph) {
        const int cj = (G * ph) / 32;   // column block of every j in this phase (G divides 32)
        const int j1 = min(G * (ph + 1), r);
        for (int j = G * ph; j < j1; ++j) {
            const int buf = j & 1;
            const int qj = j & 31;
            // owners of column j publish it (only rows > j are read)
            if (q == qj) {
#pragma unroll
                for (int m = ph; m < MR; ++m)
                    if (chol_pair<G>(m, cj)) colbuf[buf][g + G * m] = v[m][cj];
            }
            __syncthreads();
            const double piv = colbuf[buf][j];
            bad |= !(piv > 0.0);
            const double isq = 1.0 / sqrt(piv);
            const double inv = isq * isq;
            if (tid == 0) pivs[j] = piv;
            double bk[MC];
#pragma unroll
            for (int cc = cj; cc < MC; ++cc) {
                const int k = q + 32 * cc;
                const double t = colbuf[buf][k];
                bk[cc] = (k > j) ? t : 0.0;
            }
#pragma unroll
            for (int m = ph; m < MR; ++m) {
                const int i = g + G * m;
                const double t = colbuf[buf][i] * inv;
                const double am = (i > j) ? t : 0.0;
#pragma unroll
                for (int cc = cj; cc < MC; ++cc)
                    if (chol_pair<G>(m, cc)) v[m][cc] -= am * bk[cc];
            }
            if (q == qj) {
#pragma unroll
                for (int m = ph; m < MR; ++m)
                    if (chol_pair<G>(m, cj) && g + G * m >= j) v[m][cj] *= isq;
            }
        }
    }
#pragma unroll
    for (int m = 0; m < MR; ++m) {
        const int i = g + G * m;
#pragma unroll
        for (int cc = 0; cc < MC; ++cc) {
            if (chol_pair<G>(m, cc)) {
                const int k = q + 32 * cc;
                if (i < r && k <= i) a[i * r + k] = v[m][cc];
            }
        }
    }
    __syncthreads();
    double ls = 0.0;
    for (int j = tid; j < r; j += NT) ls += log(pivs[j]);
    ls = wave_sum(ls);
    if ((tid & 63) == 0) red[tid >> 6] = ls;
    const int any_bad = __syncthreads_or(bad ? 1 : 0);
    if (tid == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) t += red[w];
        if (logdet) logdet[c] = 0.5 * t;
        if (ok) ok[c] = any_bad ? 0 : 1;
    }
}

// One wave per chain for k <= 8 MB (k = 104 at MB = 13): lane (g, q) = (lane / 8, lane % 8)
// holds rows g + 8m and columns q + 8c of the lower triangle in registers (block pairs
// c <= m only, 91 doubles at MB = 13). Column j is published through LDS by its eight
// owners (q = j % 8) and read back by every lane; there is no barrier (a single wave,
// in-order LDS: wavefront-scope fences only), so a column step costs one LDS round trip
// (overlapped with the trailing update of the step before), a square root and the rank-1
// update of the lane's share of the trailing block.
template <int MB>
__global__ __launch_bounds__(64) void cholesky_wave_kernel(int r, double* A, long strideA, const int32_t* slot,
                                                           int slot_xor, long slot_stride, double* logdet,
                                                           int32_t* ok) {
    __shared__ double col[8 * MB];
    __shared__ double pivs[8 * MB];
    const int c = blockIdx.x, lane = threadIdx.x;
    const int g = lane >> 3, q = lane & 7;
    double* a = A + (long)c * strideA + slot_offset(slot, slot_xor, slot_stride, c);
    double v[MB][MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) {
        const int i = g + 8 * m;
#pragma unroll
        for (int cc = 0; cc < MB; ++cc) {
            const int kk = q + 8 * cc;
            v[m][cc] = (cc <= m && i < r && kk <= i) ? a[(long)i * r + kk] : 0.0;
        }
    }
    bool bad = false;
    if (q == 0) {  // column 0
#pragma unroll
        for (int m = 0; m < MB; ++m) col[g + 8 * m] = v[m][0];
    }
    chol_sync<true>();
    double pivot = lane_value(v[0][0], 0);
    CholWavePhases<MB, 0, true>::run(v, col, pivs, r, g, q, bad, pivot);
#pragma unroll
    for (int m = 0; m < MB; ++m) {
        const int i = g + 8 * m;
#pragma unroll
        for (int cc = 0; cc <= m; ++cc) {
            const int kk = q + 8 * cc;
            if (i < r && kk <= i) a[(long)i * r + kk] = v[m][cc];
        }
    }
    chol_sync<true>();
    double ls = 0.0;
    for (int j = lane; j < r; j += 64) ls += log(pivs[j]);
    ls = wave_sum(ls);
    const bool any_bad = __any(bad);
    if (lane == 0) {
        if (logdet) logdet[c] = 0.5 * ls;
        if (ok) ok[c] = any_bad ? 0 : 1;
    }
}

// ---------------------------------------------------------------------------------
// Reduced proposal: xp = L^-T (L^-1 [L L^T x - (1-s)(x + g)] + beta xi)
//                      = L^-T (L^T x - (1-s) L^-1 (x + g) + beta xi),
// a transposed product, a forward and a backward solve.
// lfwd (optional) = log rho_0(x -> xp) = -|xi|^2/2 + |mhat|^2/2 + logdet_x, the
// mMALA over pCN log-density ratio at the drawn point, mhat = (xp - s x)/beta.
// Chains are walked by their metadata: an idle chain is skipped, a fresh chain (one that
// joins at this step) proposes its initial state, the prior draw of stream 3, and the
// acceptance then takes it unconditionally.
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(2, 2))) void propose_kernel(int r, double s, double beta, ChainMeta meta,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ g, const double* L, long strideL,
                                                      const int32_t* slot, int slot_xor, long slot_stride,
                                                      const double* __restrict__ xi_given,
                                                      const double* __restrict__ logdet, double* __restrict__ xp,
                                                      double* __restrict__ lfwd) {
    extern __shared__ double dyn[];
    const ChainLds S = carve_chain_lds(dyn, r);
    double *xs = S.v[0], *gs = S.v[1], *xi = S.v[2], *u = S.v[3], *w = S.v[4], *t = S.v[5], *invd = S.v[6],
           *rhs = S.v[7];
    const int c = blockIdx.x, tid = threadIdx.x;
    const int32_t state = chain_state(meta, c);
    if (state == CHAIN_IDLE) return;
    if (state == CHAIN_FRESH) {
        for (int b4 = tid; 4 * b4 < r; b4 += TPB) {
            double nv[4];
            philox_normals4(meta.key0[c], meta.key1[c], (uint64_t)b4, STREAM_INIT_X, 0, (uint64_t)meta.index[c], nv);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (4 * b4 + q < r) xp[(long)c * r + 4 * b4 + q] = nv[q];
        }
        if (lfwd && tid == 0) lfwd[c] = 0.0;
        return;
    }
    const double* Lc = L + (long)c * strideL + slot_offset(slot, slot_xor, slot_stride, c);
    load_inv_diag(Lc, r, invd);
    for (int j = tid; j < r; j += TPB) {
        xs[j] = x[(long)c * r + j];
        gs[j] = g[(long)c * r + j];
        rhs[j] = xs[j] + gs[j];
    }
    if (xi_given) {
        for (int j = tid; j < r; j += TPB) xi[j] = xi_given[(long)c * r + j];
    } else {
        const uint64_t k0 = meta.key0[c], k1 = meta.key1[c];
        const uint64_t step = (uint64_t)meta.step[c], chain = (uint64_t)meta.index[c];
        for (int b4 = tid; 4 * b4 < r; b4 += TPB) {
            double nv[4];
            philox_normals4(k0, k1, (uint64_t)b4, STREAM_XI, step, chain, nv);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (4 * b4 + q < r) xi[4 * b4 + q] = nv[q];
        }
    }
    __syncthreads();
    lt_matvec2(Lc, r, xs, u, nullptr, nullptr, S.part);
    l_solve(Lc, invd, r, rhs, w, S.acc);
    for (int j = tid; j < r; j += TPB) t[j] = u[j] - (1.0 - s) * w[j] + beta * xi[j];
    __syncthreads();
    lt_solve(Lc, invd, r, t, u, S.part);
    double nxi = 0.0, nm = 0.0;
    for (int j = tid; j < r; j += TPB) {
        xp[(long)c * r + j] = u[j];
        const double m = (u[j] - s * xs[j]) / beta;
        nxi += xi[j] * xi[j];
        nm += m * m;
    }
    if (lfwd) {
        nxi = block_sum(nxi, S.red);
        nm = block_sum(nm, S.red);
        if (tid == 0) lfwd[c] = -0.5 * nxi + 0.5 * nm + logdet[c];
    }
}

// log rho_0(a -> b) with the cache (g_a, L_a, logdet_a) of a, Sec. 5.4 with
// I + H = L L^T:  -(dt/8)|L^-1 v|^2 + (sqrt(dt)/2) mhat.v - (|L^T mhat|^2 - |mhat|^2)/2
// + logdet, v = H a - g = L L^T a - a - g, mhat = (b - s a)/beta.
// Uses L^-1 v = L^T a - L^-1 (a + g) and mhat.v = (L^T mhat).(L^T a) - mhat.(a + g);
// L^T a and L^T mhat come from one pass over L. a, b, ga live in S.v[0..2].
__device__ __forceinline__ double log_rho0_dev(const double* La, int r, double dt, double s, double beta, const double* a,
                               const double* b, const double* ga, double logdet_a, const ChainLds& S) {
    const int tid = threadIdx.x;
    double *u1 = S.v[3], *w2 = S.v[4], *m = S.v[5], *u2 = S.v[6], *tmp = S.v[7], *invd = S.v[8];
    load_inv_diag(La, r, invd);
    for (int j = tid; j < r; j += TPB) {
        tmp[j] = a[j] + ga[j];
        m[j] = (b[j] - s * a[j]) / beta;
    }
    __syncthreads();
    lt_matvec2(La, r, a, u1, m, u2, S.part);
    l_solve(La, invd, r, tmp, w2, S.acc);
    double q1 = 0.0, d1 = 0.0, d2 = 0.0, n2 = 0.0, n3 = 0.0;
    for (int j = tid; j < r; j += TPB) {
        const double lv = u1[j] - w2[j];
        q1 += lv * lv;
        d1 += u2[j] * u1[j];
        d2 += m[j] * tmp[j];
        n2 += u2[j] * u2[j];
        n3 += m[j] * m[j];
    }
    q1 = block_sum(q1, S.red);
    d1 = block_sum(d1, S.red);
    d2 = block_sum(d2, S.red);
    n2 = block_sum(n2, S.red);
    n3 = block_sum(n3, S.red);
    return -(dt / 8.0) * q1 + 0.5 * sqrt(dt) * (d1 - d2) - 0.5 * (n2 - n3) + logdet_a;
}

__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(2, 2))) void log_rho_kernel(int r, double dt, double s, double beta, const double* x,
                                                      const double* phi_x, const double* g_x, const double* L_x,
                                                      const double* logdet_x, const double* xp,
                                                      const double* phi_p, const double* g_p, const double* L_p,
                                                      const double* logdet_p, double* out) {
    extern __shared__ double dyn[];
    const ChainLds S = carve_chain_lds(dyn, r);
    double *xs = S.v[0], *ps = S.v[1], *ga = S.v[2];
    const int c = blockIdx.x, tid = threadIdx.x;
    const long rr = (long)r * r;
    for (int j = tid; j < r; j += TPB) {
        xs[j] = x[(long)c * r + j];
        ps[j] = xp[(long)c * r + j];
        ga[j] = g_x[(long)c * r + j];
    }
    __syncthreads();
    const double fwd = log_rho0_dev(L_x + c * rr, r, dt, s, beta, xs, ps, ga, logdet_x[c], S);
    for (int j = tid; j < r; j += TPB) ga[j] = g_p[(long)c * r + j];
    __syncthreads();
    const double rev = log_rho0_dev(L_p + c * rr, r, dt, s, beta, ps, xs, ga, logdet_p[c], S);
    if (tid == 0) out[c] = phi_x[c] - phi_p[c] + rev - fwd;
}

// MH decision of the first stage and the swap of state and cache on acceptance.
// accflag: 0 rejected or idle, 1 accepted (pCN complement move), 2 fresh chain
// initialised (complement drawn from the prior).
// Per-step outputs of the finish: the trace (xtrace cap x C x r, phitrace cap x C; a
// chain records the step with its own step counter t as row t while t < cap; null when
// the problem keeps no trace) and the running sums of x past the burn-in (sumx; null
// outside serving). Every argument is fixed for a problem, so a captured step replays.
struct StepRecord {
    double* sumx;
    float* xtrace;
    double* phitrace;
    int64_t cap;
    int C;
};

// End of a step for chain c, run by the whole block of the accept kernels after the
// decision: the trace row, the running sum of x once the chain is past its burn-in, the
// step counter and the life cycle (a live chain that has used its step budget goes
// idle; a fresh chain becomes live). xn: the chain's state after the decision (LDS);
// step: meta.step[c] as read at the start of the kernel; phin (thread 0): the misfit
// after the decision.
__device__ __forceinline__ void finish_chain(int c, int r, const ChainMeta& meta, int32_t state, int64_t step,
                                             const double* xn, double phin, const StepRecord& rec) {
    const int tid = threadIdx.x;
    if (rec.xtrace && step < rec.cap) {
        float* xrow = rec.xtrace + step * (long)rec.C * r;
        for (int j = tid; j < r; j += TPB) xrow[(long)c * r + j] = (float)xn[j];
        if (tid == 0) rec.phitrace[step * (long)rec.C + c] = phin;
    }
    if (state == CHAIN_LIVE) {
        const int64_t s1 = step + 1;
        if (rec.sumx && s1 > meta.burn[c])
            for (int j = tid; j < r; j += TPB) rec.sumx[(long)c * r + j] += xn[j];
        if (tid == 0) {
            meta.step[c] = s1;
            if (s1 >= meta.budget[c]) meta.state[c] = CHAIN_IDLE;
        }
    } else if (state == CHAIN_FRESH && tid == 0) {
        meta.state[c] = CHAIN_LIVE;
    }
}


__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(2, 2))) void accept_kernel(int r, double dt, double s, double beta, ChainMeta meta,
                                                     double* x, double* g, double* phi,
                                                     double* logdet, const double* Lbuf, long half,
                                                     int32_t* cur, const double* xp, const double* gp,
                                                     const double* phip, const double* logdetp,
                                                     const int32_t* okp, const double* lfwd, int64_t* accepts,
                                                     int64_t* failures, int32_t* accflag, StepRecord rec, int da) {
    extern __shared__ double dyn[];
    const ChainLds S = carve_chain_lds(dyn, r);
    double *xs = S.v[0], *ps = S.v[1], *ga = S.v[2];
    __shared__ int decision;
    const int c = blockIdx.x, tid = threadIdx.x;
    const long rr = (long)r * r;
    const int32_t state = chain_state(meta, c);
    if (state == CHAIN_IDLE) {
        if (tid == 0) accflag[c] = 0;
        return;
    }
    const int64_t step = meta.step[c];  // read by every thread before the finish advances it
    double phin = 0.0;                   // thread 0: the misfit after the decision
    const int other = cur[c] ^ 1;
    const double* Lp = Lbuf + (long)other * half + c * rr;
    for (int j = tid; j < r; j += TPB) {
        xs[j] = x[(long)c * r + j];
        ps[j] = xp[(long)c * r + j];
        ga[j] = gp[(long)c * r + j];
    }
    __syncthreads();
    const int okc = okp[c];
    if (state == CHAIN_FRESH) {
        // the initial state and its cache are taken as they are
        if (tid == 0) {
            if (!okc) failures[c] += 1;
            phin = phip[c];
            phi[c] = phin;
            logdet[c] = logdetp[c];
            cur[c] = other;
            decision = 1;
            accflag[c] = 2;
        }
        __syncthreads();
    } else {
        double rev = 0.0;
        if (okc) rev = log_rho0_dev(Lp, r, dt, s, beta, ps, xs, ga, logdetp[c], S);
        if (tid == 0) {
            const double lr = phi[c] - phip[c] + rev - lfwd[c];
            const double u = philox_uniform(meta.key0[c], meta.key1[c], (uint64_t)step, (uint64_t)meta.index[c]);
            const bool good = okc && isfinite(lr);
            const bool accept = good && (log(u) <= lr);
            if (!good) failures[c] += 1;
            phin = phi[c];
            if (da) {
                // delayed acceptance: a pass goes to the second stage, which commits
                decision = 0;
                accflag[c] = accept ? 3 : 0;
            } else {
                decision = accept ? 1 : 0;
                if (accept) {
                    accepts[c] += 1;
                    phin = phip[c];
                    phi[c] = phin;
                    logdet[c] = logdetp[c];
                    cur[c] = other;
                }
                accflag[c] = decision;
            }
        }
    }
    __syncthreads();
    if (decision) {
        for (int j = tid; j < r; j += TPB) {
            x[(long)c * r + j] = ps[j];
            g[(long)c * r + j] = ga[j];
        }
    }
    if (!da) finish_chain(c, r, meta, state, step, decision ? ps : xs, phin, rec);
}

// ---------------------------------------------------------------------------------
// pCN baseline (Sec. 2.6, eq. pCN_proposal; the pCN row of the baselines of Sec. 6.1).
// In whitened coordinates the prior is N(0, I), so the proposal is x+ = s x + beta xi
// (xi: the first r normals of the proposal stream, as the mMALA proposal draws them), and
// prior reversibility makes the transition rate ratio exp(Phi(x) - Phi(x+)). No Jacobian,
// metric or factor is formed: a step is this proposal, the network forward at x+ and the
// decision kernel below. One wave per chain; a fresh chain (serving life cycle) draws its
// initial state from the prior as the mMALA proposal kernel does.
__global__ __launch_bounds__(64) void pcn_propose_kernel(int r, double s, double beta, ChainMeta meta,
                                                         const double* __restrict__ x, double* __restrict__ xp) {
    const int c = blockIdx.x, lane = threadIdx.x;
    const int32_t state = chain_state(meta, c);
    if (state == CHAIN_IDLE) return;
    const bool fresh = state == CHAIN_FRESH;
    const uint64_t k0 = meta.key0[c], k1 = meta.key1[c], chain = (uint64_t)meta.index[c];
    const uint64_t stream = fresh ? STREAM_INIT_X : STREAM_XI, step = fresh ? 0 : (uint64_t)meta.step[c];
    for (int b4 = lane; 4 * b4 < r; b4 += 64) {
        double nv[4];
        philox_normals4(k0, k1, (uint64_t)b4, stream, step, chain, nv);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * b4 + q;
            if (j < r) xp[(long)c * r + j] = fresh ? nv[q] : s * x[(long)c * r + j] + beta * nv[q];
        }
    }
}

// LA-pCN proposal (eq. MAP and the LA-pCN proposal after it, with the mean read as
// x_map + s (x - x_map)): x+ = x_map + s (x - x_map) + beta L^-T xi, L the fixed factor
// of I + H(x_map) shared by every chain. lterm receives the density part of log rho,
// (|x|^2 - |x+|^2)/2 + (|L^T (x+ - x_map)|^2 - |L^T (x - x_map)|^2)/2; the decision
// kernel adds Phi(x) - Phi(x+). One block per chain.
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(2, 2))) void lapcn_propose_kernel(
    int r, double s, double beta, ChainMeta meta, const double* __restrict__ x, const double* L,
    const double* __restrict__ xmap, double* __restrict__ xp, double* __restrict__ lterm) {
    extern __shared__ double dyn[];
    const ChainLds S = carve_chain_lds(dyn, r);
    double *xi = S.v[0], *u = S.v[1], *dx = S.v[2], *dp = S.v[3], *lx = S.v[4], *lp = S.v[5], *invd = S.v[6];
    const int c = blockIdx.x, tid = threadIdx.x;
    const int32_t state = chain_state(meta, c);
    if (state == CHAIN_IDLE) return;
    const uint64_t k0 = meta.key0[c], k1 = meta.key1[c], chain = (uint64_t)meta.index[c];
    if (state == CHAIN_FRESH) {
        for (int b4 = tid; 4 * b4 < r; b4 += TPB) {
            double nv[4];
            philox_normals4(k0, k1, (uint64_t)b4, STREAM_INIT_X, 0, chain, nv);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (4 * b4 + q < r) xp[(long)c * r + 4 * b4 + q] = nv[q];
        }
        if (tid == 0) lterm[c] = 0.0;
        return;
    }
    load_inv_diag(L, r, invd);
    const uint64_t step = (uint64_t)meta.step[c];
    for (int b4 = tid; 4 * b4 < r; b4 += TPB) {
        double nv[4];
        philox_normals4(k0, k1, (uint64_t)b4, STREAM_XI, step, chain, nv);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (4 * b4 + q < r) xi[4 * b4 + q] = nv[q];
    }
    __syncthreads();
    lt_solve(L, invd, r, xi, u, S.part);
    __syncthreads();
    double nx = 0.0, np = 0.0;
    for (int j = tid; j < r; j += TPB) {
        const double xj = x[(long)c * r + j], mj = xmap[j];
        const double pj = mj + s * (xj - mj) + beta * u[j];
        xp[(long)c * r + j] = pj;
        dx[j] = xj - mj;
        dp[j] = pj - mj;
        nx += xj * xj;
        np += pj * pj;
    }
    __syncthreads();
    lt_matvec2(L, r, dx, lx, dp, lp, S.part);
    __syncthreads();
    double qx = 0.0, qp = 0.0;
    for (int j = tid; j < r; j += TPB) {
        qx += lx[j] * lx[j];
        qp += lp[j] * lp[j];
    }
    nx = block_sum(nx, S.red);
    np = block_sum(np, S.red);
    qx = block_sum(qx, S.red);
    qp = block_sum(qp, S.red);
    if (tid == 0) lterm[c] = 0.5 * (nx - np) + 0.5 * (qp - qx);
}

// Misfit at x+ (Sec. 5.1: 1/2 || Gamma^-1/2 (f - y) ||^2, from the network output f of
// the forward stage, FP64 or FP32), the MH decision with exp(Phi(x) - Phi(x+)) (accept iff
// log u <= log rho; a non-finite misfit rejects and is counted) and the end of the step.
// lterm (LA-pCN): the density part of log rho from the proposal kernel, or null (pCN).
// accflag as for the mMALA accept kernel (the complement kernel reads it).
template <typename TF>
__global__ __launch_bounds__(TPB) void pcn_accept_kernel(int r, int dy, ChainMeta meta, const TF* __restrict__ f,
                                                         const double* __restrict__ y_rows,
                                                         const double* __restrict__ winv_rows, double* x,
                                                         double* phi, const double* __restrict__ xp,
                                                         const double* __restrict__ lterm, int64_t* accepts,
                                                         int64_t* failures, int32_t* accflag, StepRecord rec) {
    __shared__ double red[TPB / 64];
    __shared__ int decision;
    const int c = blockIdx.x, tid = threadIdx.x;
    const int32_t state = chain_state(meta, c);
    if (state == CHAIN_IDLE) {
        if (tid == 0) accflag[c] = 0;
        return;
    }
    const int64_t step = meta.step[c];  // read by every thread before the finish advances it
    const long row = chain_row(meta, c);
    const double* y = y_rows + row * dy;
    const double* winv = winv_rows + row * dy;
    double part = 0.0;
    for (int i = tid; i < dy; i += TPB) {
        const double w = winv[i];
        const double v = (w == 0.0) ? 0.0 : ((double)f[(long)c * dy + i] - y[i]) * w;
        part += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if ((tid & 63) == 0) red[tid >> 6] = part;
    __syncthreads();
    double phin = 0.0;  // thread 0: the misfit after the decision
    if (tid == 0) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < TPB / 64; ++k) t += red[k];
        const double php = 0.5 * t;
        if (state == CHAIN_FRESH) {
            // the initial state is taken as it is
            if (!isfinite(php)) failures[c] += 1;
            phin = php;
            phi[c] = php;
            decision = 1;
            accflag[c] = 2;
        } else {
            const double lr = phi[c] - php + (lterm ? lterm[c] : 0.0);
            const double u = philox_uniform(meta.key0[c], meta.key1[c], (uint64_t)step, (uint64_t)meta.index[c]);
            const bool good = isfinite(lr);
            const bool accept = good && (log(u) <= lr);
            if (!good) failures[c] += 1;
            phin = phi[c];
            if (accept) {
                accepts[c] += 1;
                phin = php;
                phi[c] = php;
            }
            decision = accept ? 1 : 0;
            accflag[c] = decision;
        }
    }
    __syncthreads();
    const double* xn = (decision ? xp : x) + (long)c * r;
    if (decision)
        for (int j = tid; j < r; j += TPB) x[(long)c * r + j] = xp[(long)c * r + j];
    finish_chain(c, r, meta, state, step, xn, phin, rec);
}

// ---------------------------------------------------------------------------------
// MALA baseline (the MALA row of the baselines of Sec. 6.1: the ppg, no metric). It is the
// mMALA transition with H = 0: x+ = s x - (1 - s) g + beta xi, and the RN derivative with
// respect to pCN keeps its ppg terms only,
//   log rho_0(m1, m2) = -(dt/8) ||g(m1)||^2 - (sqrt(dt)/2) mhat . g(m1),
//   mhat = (m2 - s m1) / beta.
// The geometry stages still form the misfit and ppg at x+ (Jacobian sweep included); no
// factor is formed or used.
// One wave per chain: the proposal and the forward term log rho_0(x -> x+) (into lfwd).
// With lam (DIS-mMALA: the fixed metric diag(lam) of eq. dis_gnh in DIS coordinates) the
// proposal is x+_j = ((lam_j + s) x_j - (1 - s) g_j)/(1 + lam_j) + beta xi_j / sqrt(1 + lam_j)
// and, with v = lam a - g(a), log rho_0(a, b) = -(dt/8) sum v_j^2/(1 + lam_j) +
// (sqrt(dt)/2) mhat . v - (1/2) sum lam_j mhat_j^2 (its log det term cancels in the ratio).
__global__ __launch_bounds__(64) void mala_propose_kernel(int r, double dt, double s, double beta, ChainMeta meta,
                                                          const double* __restrict__ x,
                                                          const double* __restrict__ g, double* __restrict__ xp,
                                                          double* __restrict__ lfwd, const double* __restrict__ lam) {
    const int c = blockIdx.x, lane = threadIdx.x;
    const int32_t state = chain_state(meta, c);
    if (state == CHAIN_IDLE) return;
    const bool fresh = state == CHAIN_FRESH;
    const uint64_t k0 = meta.key0[c], k1 = meta.key1[c], chain = (uint64_t)meta.index[c];
    const uint64_t stream = fresh ? STREAM_INIT_X : STREAM_XI, step = fresh ? 0 : (uint64_t)meta.step[c];
    double gg = 0.0, mg = 0.0, hm = 0.0;
    for (int b4 = lane; 4 * b4 < r; b4 += 64) {
        double nv[4];
        philox_normals4(k0, k1, (uint64_t)b4, stream, step, chain, nv);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * b4 + q;
            if (j >= r) continue;
            if (fresh) {
                xp[(long)c * r + j] = nv[q];
                continue;
            }
            const double xj = x[(long)c * r + j], gj = g[(long)c * r + j];
            if (lam) {
                const double lj = lam[j], d1 = 1.0 + lj;
                const double pj = ((lj + s) * xj - (1.0 - s) * gj) / d1 + beta * nv[q] / sqrt(d1);
                xp[(long)c * r + j] = pj;
                const double vj = lj * xj - gj, mj = (pj - s * xj) / beta;
                gg += vj * vj / d1;
                mg -= mj * vj;
                hm += lj * mj * mj;
            } else {
                const double pj = s * xj - (1.0 - s) * gj + beta * nv[q];
                xp[(long)c * r + j] = pj;
                gg += gj * gj;
                mg += ((pj - s * xj) / beta) * gj;
            }
        }
    }
    gg = wave_sum(gg);
    mg = wave_sum(mg);
    hm = wave_sum(hm);
    if (lane == 0) lfwd[c] = fresh ? 0.0 : -(dt / 8.0) * gg - (sqrt(dt) / 2.0) * mg - 0.5 * hm;
}

// The reverse term log rho_0(x+ -> x) with the ppg at x+, the MH decision (a non-finite
// misfit or ppg rejects and is counted) and the end of the step; x, g and phi follow the
// decision. accflag as for the mMALA accept kernel.
__global__ __launch_bounds__(TPB) void mala_accept_kernel(int r, double dt, double s, double beta, ChainMeta meta,
                                                          double* x, double* g, double* phi,
                                                          const double* __restrict__ xp,
                                                          const double* __restrict__ gp,
                                                          const double* __restrict__ phip,
                                                          const double* __restrict__ lfwd, int64_t* accepts,
                                                          int64_t* failures, int32_t* accflag, StepRecord rec,
                                                          const double* __restrict__ lam) {
    __shared__ double red[3][TPB / 64];
    __shared__ int decision;
    const int c = blockIdx.x, tid = threadIdx.x;
    const int32_t state = chain_state(meta, c);
    if (state == CHAIN_IDLE) {
        if (tid == 0) accflag[c] = 0;
        return;
    }
    const int64_t step = meta.step[c];  // read by every thread before the finish advances it
    double gg = 0.0, mg = 0.0, hm = 0.0;
    for (int j = tid; j < r; j += TPB) {
        const double gj = gp[(long)c * r + j], pj = xp[(long)c * r + j];
        if (lam) {
            const double lj = lam[j], vj = lj * pj - gj, mj = (x[(long)c * r + j] - s * pj) / beta;
            gg += vj * vj / (1.0 + lj);
            mg -= mj * vj;
            hm += lj * mj * mj;
        } else {
            gg += gj * gj;
            mg += ((x[(long)c * r + j] - s * pj) / beta) * gj;
        }
    }
    gg = wave_sum(gg);
    mg = wave_sum(mg);
    hm = wave_sum(hm);
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = gg;
        red[1][tid >> 6] = mg;
        red[2][tid >> 6] = hm;
    }
    __syncthreads();
    double phin = 0.0;  // thread 0: the misfit after the decision
    if (tid == 0) {
        double sg = 0.0, sm = 0.0, sh = 0.0;
#pragma unroll
        for (int k = 0; k < TPB / 64; ++k) {
            sg += red[0][k];
            sm += red[1][k];
            sh += red[2][k];
        }
        const double php = phip[c];
        if (state == CHAIN_FRESH) {
            if (!isfinite(php) || !isfinite(sg)) failures[c] += 1;
            phin = php;
            phi[c] = php;
            decision = 1;
            accflag[c] = 2;
        } else {
            const double rev = -(dt / 8.0) * sg - (sqrt(dt) / 2.0) * sm - 0.5 * sh;
            const double lr = phi[c] - php + rev - lfwd[c];
            const double u = philox_uniform(meta.key0[c], meta.key1[c], (uint64_t)step, (uint64_t)meta.index[c]);
            const bool good = isfinite(lr);
            const bool accept = good && (log(u) <= lr);
            if (!good) failures[c] += 1;
            phin = phi[c];
            if (accept) {
                accepts[c] += 1;
                phin = php;
                phi[c] = php;
            }
            decision = accept ? 1 : 0;
            accflag[c] = decision;
        }
    }
    __syncthreads();
    if (decision)
        for (int j = tid; j < r; j += TPB) {
            x[(long)c * r + j] = xp[(long)c * r + j];
            g[(long)c * r + j] = gp[(long)c * r + j];
        }
    finish_chain(c, r, meta, state, step, (decision ? xp : x) + (long)c * r, phin, rec);
}

// ---------------------------------------------------------------------------------
// Observation-space (dual) form for d_y < r. With B = Gamma^-1/2 J (d_y x r) and the
// Cholesky factor K of M = I + B B^T (d_y x d_y), (I + H)^-1 v = v - B^T M^-1 B v
// (Woodbury), log det (I + H) = log det M, and the proposal noise is drawn as
// beta (I + H)^-1 (xi_1 + B^T xi_2) (xi_1 in R^r, xi_2 in R^d_y: the first r and the
// next d_y normals of the proposal stream), which has covariance beta^2 (I + H)^-1.

// y_i = sum_j B[i][j] v_j (i < dy): one wave per row, lanes over j.
template <typename TB>
__device__ __forceinline__ void b_times(const TB* __restrict__ B, int dy, int r, int ldb, const double* v, double* y) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = wave; i < dy; i += TPB / 64) {
        double acc = 0.0;
        for (int j = lane; j < r; j += 64) acc += to_d(B[(long)i * ldb + j]) * v[j];
        acc = wave_sum(acc);
        if (lane == 0) y[i] = acc;
    }
    __syncthreads();
}

// w_j = sum_i B[i][j] z_i (j < r): threads over j.
template <typename TB>
__device__ __forceinline__ void bt_times(const TB* __restrict__ B, int dy, int r, int ldb, const double* z, double* w) {
    for (int j = threadIdx.x; j < r; j += TPB) {
        double acc = 0.0;
#pragma unroll 4
        for (int i = 0; i < dy; ++i) acc += to_d(B[(long)i * ldb + j]) * z[i];
        w[j] = acc;
    }
    __syncthreads();
}

// BF16 B staged in LDS (row stride ldl = ldb + 8: rows 16 bytes apart in bank order, so
// that the 16-byte row reads of b_times from 32 rows spread over the banks; columns
// r..ldb are zero). Two BF16 values of a 32-bit word, as doubles (exact).
__device__ __forceinline__ double bf_lo(uint32_t u) { return (double)__uint_as_float(u << 16); }
__device__ __forceinline__ double bf_hi(uint32_t u) { return (double)__uint_as_float(u & 0xFFFF0000u); }

// y_i = sum_{j<r} B[i][j] v_j and, if TWO, y2_i = sum_j B[i][j] v2_j, B in LDS. P
// consecutive threads share a row, each taking every P-th 16-byte chunk of it; the P
// partial sums meet by xor shuffles inside the wave (no per-row reduction over 64 lanes).
template <int NV>
__device__ __forceinline__ void b_times_lds(const __hip_bfloat16* B, int dy, int r, int ldl, const double* const (&vs)[NV],
                                            double* const (&ys)[NV]) {
    const int nfull = r >> 3, nch = (r + 7) >> 3;
    int P = 1;
    while (P < 8 && 2 * P * dy <= TPB && 2 * P <= nch) P *= 2;
    for (int t0 = 0; t0 < dy * P; t0 += TPB) {
        const int t = t0 + (int)threadIdx.x;
        const int i = t / P, p = t & (P - 1);
        double a0[NV], a1[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) a0[q] = a1[q] = 0.0;
        if (i < dy) {
            const uint4* row = reinterpret_cast<const uint4*>(B + (long)i * ldl);
            int kq = p;
            // full chunks two at a time: both chunks' LDS reads before the products
            for (; kq + P < nfull; kq += 2 * P) {
                const uint4 qa = row[kq], qb = row[kq + P];
                double va[NV][8], vb[NV][8];
#pragma unroll
                for (int q = 0; q < NV; ++q)
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        va[q][e] = vs[q][8 * kq + e];
                        vb[q][e] = vs[q][8 * (kq + P) + e];
                    }
                const uint32_t wa[4] = {qa.x, qa.y, qa.z, qa.w}, wb[4] = {qb.x, qb.y, qb.z, qb.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double blo = bf_lo(wa[e]), bhi = bf_hi(wa[e]);
#pragma unroll
                    for (int q = 0; q < NV; ++q) {
                        a0[q] += blo * va[q][2 * e];
                        a1[q] += bhi * va[q][2 * e + 1];
                    }
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double blo = bf_lo(wb[e]), bhi = bf_hi(wb[e]);
#pragma unroll
                    for (int q = 0; q < NV; ++q) {
                        a0[q] += blo * vb[q][2 * e];
                        a1[q] += bhi * vb[q][2 * e + 1];
                    }
                }
            }
            for (; kq < nch; kq += P) {
                const uint4 qv = row[kq];
                const uint32_t w4[4] = {qv.x, qv.y, qv.z, qv.w};
                if (kq < nfull) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const double blo = bf_lo(w4[e]), bhi = bf_hi(w4[e]);
#pragma unroll
                        for (int q = 0; q < NV; ++q) {
                            a0[q] += blo * vs[q][8 * kq + 2 * e];
                            a1[q] += bhi * vs[q][8 * kq + 2 * e + 1];
                        }
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const double blo = bf_lo(w4[e]), bhi = bf_hi(w4[e]);
#pragma unroll
                        for (int q = 0; q < NV; ++q) {
                            if (8 * kq + 2 * e < r) a0[q] += blo * vs[q][8 * kq + 2 * e];
                            if (8 * kq + 2 * e + 1 < r) a1[q] += bhi * vs[q][8 * kq + 2 * e + 1];
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double acc = a0[q] + a1[q];
            for (int o = 1; o < P; o <<= 1) acc += __shfl_xor(acc, o);
            if (i < dy && p == 0) ys[q][i] = acc;
        }
    }
    __syncthreads();
}

// w_j = sum_i B[i][j] z_i (j < r) and, if w2, w2 = B^T z2 in the same pass, B in LDS: a
// thread takes a column pair (4-byte reads, consecutive across lanes) and every Q-th
// row; the Q row shares are added in turn.
__device__ __forceinline__ void bt_times_lds(const __hip_bfloat16* B, int dy, int r, int ldl, const double* z, double* w,
                                             const double* z2 = nullptr, double* w2 = nullptr) {
    const int np = (r + 1) >> 1;
    const int Q = max(1, min(TPB / np, dy));
    const int tid = threadIdx.x, jp = tid % np, q = tid / np;
    const bool act = q < Q;
    double a0 = 0.0, a1 = 0.0, c0 = 0.0, c1 = 0.0;
    if (act) {
        // U rows per batch: their LDS reads are issued before the products
        constexpr int U = 8;
        int i = q;
        for (; i + (U - 1) * Q < dy; i += U * Q) {
            uint32_t uu[U];
            double zz[U], zz2[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                uu[k] = *reinterpret_cast<const uint32_t*>(B + (long)(i + k * Q) * ldl + 2 * jp);
                zz[k] = z[i + k * Q];
                if (z2) zz2[k] = z2[i + k * Q];
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                a0 += bf_lo(uu[k]) * zz[k];
                a1 += bf_hi(uu[k]) * zz[k];
                if (z2) {
                    c0 += bf_lo(uu[k]) * zz2[k];
                    c1 += bf_hi(uu[k]) * zz2[k];
                }
            }
        }
        for (; i < dy; i += Q) {
            const uint32_t u = *reinterpret_cast<const uint32_t*>(B + (long)i * ldl + 2 * jp);
            const double zi = z[i];
            a0 += bf_lo(u) * zi;
            a1 += bf_hi(u) * zi;
            if (z2) {
                const double z2i = z2[i];
                c0 += bf_lo(u) * z2i;
                c1 += bf_hi(u) * z2i;
            }
        }
    }
    const int j = 2 * jp;
    for (int qq = 0; qq < Q; ++qq) {
        if (act && q == qq) {
            w[j] = (qq == 0 ? 0.0 : w[j]) + a0;
            if (j + 1 < r) w[j + 1] = (qq == 0 ? 0.0 : w[j + 1]) + a1;
            if (w2) {
                w2[j] = (qq == 0 ? 0.0 : w2[j]) + c0;
                if (j + 1 < r) w2[j + 1] = (qq == 0 ? 0.0 : w2[j + 1]) + c1;
            }
        }
        __syncthreads();
    }
}

// The BF16 instances read B from LDS (staged with row stride ldl).
__device__ __forceinline__ void b_times(const __hip_bfloat16* B, int dy, int r, int ldl, const double* v, double* y) {
    const double* const vs[1] = {v};
    double* const ys[1] = {y};
    b_times_lds<1>(B, dy, r, ldl, vs, ys);
}
__device__ __forceinline__ void bt_times(const __hip_bfloat16* B, int dy, int r, int ldl, const double* z, double* w) {
    bt_times_lds(B, dy, r, ldl, z, w);
}
// w = B^T z and w2 = B^T z2 in one pass over B
__device__ __forceinline__ void bt_times2(const __hip_bfloat16* B, int dy, int r, int ldl, const double* z, double* w,
                                          const double* z2, double* w2) {
    bt_times_lds(B, dy, r, ldl, z, w, z2, w2);
}
__device__ __forceinline__ void bt_times2(const double* B, int dy, int r, int ldb, const double* z, double* w,
                                          const double* z2, double* w2) {
    bt_times(B, dy, r, ldb, z, w);
    bt_times(B, dy, r, ldb, z2, w2);
}
// y = B v and y2 = B v2 in one pass over B
__device__ __forceinline__ void b_times2(const __hip_bfloat16* B, int dy, int r, int ldl, const double* v, double* y,
                                         const double* v2, double* y2) {
    const double* const vs[2] = {v, v2};
    double* const ys[2] = {y, y2};
    b_times_lds<2>(B, dy, r, ldl, vs, ys);
}
__device__ __forceinline__ void b_times2(const double* B, int dy, int r, int ldb, const double* v, double* y,
                                         const double* v2, double* y2) {
    b_times(B, dy, r, ldb, v, y);
    b_times(B, dy, r, ldb, v2, y2);
}
// y_q = B v_q for three vectors in one pass over B
__device__ __forceinline__ void b_times3(const __hip_bfloat16* B, int dy, int r, int ldl, const double* v1,
                                         double* y1, const double* v2, double* y2, const double* v3, double* y3) {
    const double* const vs[3] = {v1, v2, v3};
    double* const ys[3] = {y1, y2, y3};
    b_times_lds<3>(B, dy, r, ldl, vs, ys);
}
__device__ __forceinline__ void b_times3(const double* B, int dy, int r, int ldb, const double* v1, double* y1,
                                         const double* v2, double* y2, const double* v3, double* y3) {
    b_times(B, dy, r, ldb, v1, y1);
    b_times(B, dy, r, ldb, v2, y2);
    b_times(B, dy, r, ldb, v3, y3);
}

// Scratch of the dual kernels: vectors of length r and d_y in dynamic LDS, followed
// (BF16 path) by the chain's B (d_y x ldl), staged once so that every product reads LDS.
constexpr int DU_NR = 8, DU_NY = 8;
constexpr int DU_RED = 4 * (TPB / 64);  // block_sum4 scratch
__host__ __device__ inline int dual_ldl(int ldb, bool stage_bf16) { return stage_bf16 ? ldb + 8 : ldb; }
__host__ __device__ inline size_t dual_lds_doubles(int r, int dy, int ldb, bool stage_bf16) {
    const size_t b = stage_bf16 ? ((size_t)dy * dual_ldl(ldb, true) * sizeof(__hip_bfloat16) + 7) / 8 : 0;
    return (size_t)DU_NR * r + (size_t)DU_NY * dy + SB + (size_t)8 * SB + DU_RED + (size_t)8 * SB + b;
}

// BF16 B rows are copied to LDS (16-byte moves, row stride ldb + 8) and used from there;
// FP64 B is read from global memory as it is.
// sync = false leaves the barrier to the caller (other loads can share its round trip).
__device__ __forceinline__ const double* stage_b(const double* Bg, int, int, double*, bool = true) { return Bg; }
__device__ __forceinline__ const __hip_bfloat16* stage_b(const __hip_bfloat16* Bg, int dy, int ldb, double* lds,
                                                          bool sync = true) {
    __hip_bfloat16* Bl = reinterpret_cast<__hip_bfloat16*>(lds);
    const int c16 = ldb / 8, l16 = dual_ldl(ldb, true) / 8;  // 16-byte chunks per row (ldb: a multiple of 32)
    const int n16 = dy * c16;
    const uint4* src = reinterpret_cast<const uint4*>(Bg);
    uint4* dst = reinterpret_cast<uint4*>(Bl);
    // SBATCH chunks per thread in flight: the loads of a batch go out before its LDS stores
    constexpr int SBATCH = 4;
    for (int base = 0; base < n16; base += SBATCH * TPB) {
        uint4 v[SBATCH];
#pragma unroll
        for (int u = 0; u < SBATCH; ++u) {
            const int e = base + u * TPB + (int)threadIdx.x;
            v[u] = make_uint4(0u, 0u, 0u, 0u);
            if (e < n16) v[u] = src[e];
        }
#pragma unroll
        for (int u = 0; u < SBATCH; ++u) {
            const int e = base + u * TPB + (int)threadIdx.x;
            const int row = e / c16;
            if (e < n16) dst[row * l16 + (e - row * c16)] = v[u];
        }
    }
    if (sync) __syncthreads();
    return Bl;
}

// log rho_0(a -> b) (Sec. 5.4) with the cache (g_a, B_a, K_a, logdet_a) of a:
//   -(dt/8) v^T (I + H)^-1 v + (sqrt(dt)/2) mhat^T v - mhat^T H mhat / 2 + logdet,
// v = H a - g_a, mhat = (b - s a)/beta, with v^T (I + H)^-1 v = |v|^2 - |K^-1 B v|^2 and
// mhat^T H mhat = |B mhat|^2. Vectors in R: v, mh, and in Y: t1, t2, z.
template <typename TB>
__device__ __forceinline__ double dual_rho0(const TB* Ba, int ldb, const double* Ka, const double* invd, int r, int dy, double dt,
                            double s, double beta, const double* a, const double* b, const double* ga,
                            double logdet_a, double* v, double* mh, double* t1, double* t2, double* z,
                            double* acc_s, double* red, int dinv) {
    const int tid = threadIdx.x;
    b_times(Ba, dy, r, ldb, a, t1);
    bt_times(Ba, dy, r, ldb, t1, v);
    for (int j = tid; j < r; j += TPB) {
        v[j] -= ga[j];
        mh[j] = (b[j] - s * a[j]) / beta;
    }
    __syncthreads();
    b_times2(Ba, dy, r, ldb, v, t2, mh, t1);
    if (dinv) l_solve_dinv(Ka, invd, dy, t2, z, nullptr, nullptr, acc_s);
    else l_solve(Ka, invd, dy, t2, z, acc_s);
    double sums[4] = {0.0, 0.0, 0.0, 0.0};  // |v|^2, mh.v, |z|^2, |B mh|^2
    for (int j = tid; j < r; j += TPB) {
        sums[0] += v[j] * v[j];
        sums[1] += mh[j] * v[j];
    }
    for (int i = tid; i < dy; i += TPB) {
        sums[2] += z[i] * z[i];
        sums[3] += t1[i] * t1[i];
    }
    block_sum4(sums, red);
    return -(dt / 8.0) * (sums[0] - sums[2]) + 0.5 * sqrt(dt) * sums[1] - 0.5 * sums[3] + logdet_a;
}

// Proposal: u = beta (xi_1 + B^T xi_2) - (1 - s)(x + g),  xp = x + (I + H)^-1 u,
// and lfwd = log rho_0(x -> xp) with the cache of x. B: the state's B (C x dy x ldb).
// xi_given (n x (r + dy), xi_1 then xi_2) replaces the Philox draws when not null.
template <typename TB>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(2, 2)))
void propose_dual_kernel(int r, int dy, int ldb, double dt, double s, double beta, ChainMeta meta,
                         const double* __restrict__ x, const double* __restrict__ g, const TB* __restrict__ B,
                         const double* Kbuf, long strideK, const int32_t* slot, int slot_xor, long slot_stride,
                         const double* __restrict__ logdet, const double* __restrict__ xi_given,
                         double* __restrict__ xp, double* __restrict__ lfwd, int dinv) {
    extern __shared__ double dyn[];
    double* R = dyn;
    double *xs = R, *gs = R + r, *u = R + 2 * r, *w = R + 3 * r, *v = R + 4 * r, *mh = R + 5 * r,
           *xi1 = R + 6 * r, *xn = R + 7 * r;
    double* Y = dyn + (size_t)DU_NR * r;
    double *xi2 = Y, *y = Y + dy, *z1 = Y + 2 * dy, *invd = Y + 3 * dy, *t1 = Y + 4 * dy, *t2 = Y + 5 * dy;
    double* acc = Y + (size_t)DU_NY * dy;
    double* part = acc + SB;
    double* red = part + 8 * SB;
    const int c = blockIdx.x, tid = threadIdx.x;
    const int32_t state = chain_state(meta, c);
    if (state == CHAIN_IDLE) return;
    if (state == CHAIN_FRESH) {
        for (int b4 = tid; 4 * b4 < r; b4 += TPB) {
            double nv[4];
            philox_normals4(meta.key0[c], meta.key1[c], (uint64_t)b4, STREAM_INIT_X, 0, (uint64_t)meta.index[c], nv);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (4 * b4 + q < r) xp[(long)c * r + 4 * b4 + q] = nv[q];
        }
        if (lfwd && tid == 0) lfwd[c] = 0.0;
        return;
    }
    // B's staging, the pivots' reciprocals, the states and the draws share one barrier
    double* part2 = red + DU_RED;  // 8 SB doubles: the partial sums of K^T (B x) in the back solve
    const TB* Bc = stage_b(B + (long)c * dy * ldb, dy, ldb, part2 + 8 * SB, false);
    const int ldl = dual_ldl(ldb, sizeof(TB) == 2);  // row stride of Bc
    const double* Kc = Kbuf + (long)c * strideK + slot_offset(slot, slot_xor, slot_stride, c);
    load_inv_diag(Kc, dy, invd, false);
    for (int j = tid; j < r; j += TPB) {
        xs[j] = x[(long)c * r + j];
        gs[j] = g[(long)c * r + j];
    }
    if (xi_given) {
        for (int k = tid; k < r + dy; k += TPB) {
            const double v = xi_given[(long)c * (r + dy) + k];
            if (k < r) xi1[k] = v;
            else xi2[k - r] = v;
        }
    } else {
        const uint64_t k0 = meta.key0[c], k1 = meta.key1[c];
        const uint64_t step = (uint64_t)meta.step[c], chain = (uint64_t)meta.index[c];
        for (int b4 = tid; 4 * b4 < r + dy; b4 += TPB) {
            double nv[4];
            philox_normals4(k0, k1, (uint64_t)b4, STREAM_XI, step, chain, nv);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 4 * b4 + q;
                if (k < r) xi1[k] = nv[q];
                else if (k < r + dy) xi2[k - r] = nv[q];
            }
        }
    }
    __syncthreads();
    bt_times(Bc, dy, r, ldl, xi2, w);
    for (int j = tid; j < r; j += TPB) u[j] = beta * (xi1[j] + w[j]) - (1.0 - s) * (xs[j] + gs[j]);
    __syncthreads();
    // y = B u, and B x, B g for the forward term (xi2 is free: it holds B g)
    double *bx = Y + 6 * dy, *zs = Y + 7 * dy, *bg = xi2;
    b_times3(Bc, dy, r, ldl, u, y, xs, bx, gs, bg);
    for (int i = tid; i < dy; i += TPB) t2[i] = bx[i] + bg[i];
    __syncthreads();
    // z1 = K^-1 B u and zs = K^-1 B (x + g) in one sweep
    // with the inverted blocks the back solve also forms K^T (B x) (into bg: B g is spent),
    // the forward term's product
    double* kbx = bg;
    if (dinv) {
        l_solve_dinv(Kc, invd, dy, y, z1, t2, zs, part);
        lt_solve_dinv(Kc, invd, dy, z1, t1, part, acc, lfwd ? bx : nullptr, kbx, part2);
    } else {
        l_solve2(Kc, invd, dy, y, z1, t2, zs, part);
        lt_solve(Kc, invd, dy, z1, t1, part);
    }
    // w = B^T t1 and, for the forward term, v = B^T (B x) in the same pass over B
    if (lfwd) bt_times2(Bc, dy, r, ldl, t1, w, bx, v);
    else bt_times(Bc, dy, r, ldl, t1, w);
    for (int j = tid; j < r; j += TPB) {
        xn[j] = xs[j] + u[j] - w[j];
        xp[(long)c * r + j] = xn[j];
        if (lfwd) {
            v[j] -= gs[j];
            mh[j] = (xn[j] - s * xs[j]) / beta;
        }
    }
    __syncthreads();
    if (lfwd) {
        // log rho_0(x -> xn) with the cache of x (the reverse term of the dual form):
        // v = H x - g = B^T (B x) - g, and K^-1 B v = K^T (B x) - K^-1 B (x + g), since
        // B B^T = K K^T - I; the second term is zs from the sweep above.
        b_times(Bc, dy, r, ldl, mh, y);          // y = B mhat
        if (!dinv) lt_matvec(Kc, dy, bx, kbx, part);  // K^T (B x)
        double sums[4] = {0.0, 0.0, 0.0, 0.0};   // |v|^2, mhat.v, |K^-1 B v|^2, |B mhat|^2
        for (int j = tid; j < r; j += TPB) {
            sums[0] += v[j] * v[j];
            sums[1] += mh[j] * v[j];
        }
        for (int i = tid; i < dy; i += TPB) {
            const double zr = kbx[i] - zs[i];
            sums[2] += zr * zr;
            sums[3] += y[i] * y[i];
        }
        block_sum4(sums, red);
        const double l = -(dt / 8.0) * (sums[0] - sums[2]) + 0.5 * sqrt(dt) * sums[1] - 0.5 * sums[3] + logdet[c];
        if (tid == 0) lfwd[c] = l;
    }
}

// MH decision of the dual form: reverse term with the proposal's cache (B of the
// proposal, its factor in the other half of Kbuf); on acceptance the proposal's B
// becomes the state's (copied), the factor half flips.
template <typename TB>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(2, 2)))
void accept_dual_kernel(int r, int dy, int ldb, double dt, double s, double beta, ChainMeta meta, double* x, double* g,
                        double* phi, double* logdet, const double* Kbuf, long half, int32_t* cur, const double* xp,
                        const double* gp, const double* phip, const double* logdetp, const int32_t* okp,
                        const double* lfwd, const TB* __restrict__ Bp, TB* __restrict__ Bs, int64_t* accepts,
                        int64_t* failures, int32_t* accflag, StepRecord rec, int da, int dinv) {
    extern __shared__ double dyn[];
    double* R = dyn;
    double *xs = R, *ps = R + r, *ga = R + 2 * r, *v = R + 3 * r, *mh = R + 4 * r;
    double* Y = dyn + (size_t)DU_NR * r;
    double *invd = Y, *t1 = Y + dy, *t2 = Y + 2 * dy, *z = Y + 3 * dy;
    double* acc = Y + (size_t)DU_NY * dy;
    double* red = acc + 9 * SB;
    __shared__ int decision;
    const int c = blockIdx.x, tid = threadIdx.x;
    const long kk = (long)dy * dy;
    const int32_t state = chain_state(meta, c);
    if (state == CHAIN_IDLE) {
        if (tid == 0) accflag[c] = 0;
        return;
    }
    const int64_t step = meta.step[c];  // read by every thread before the finish advances it
    double phin = 0.0;                   // thread 0: the misfit after the decision
    const int other = cur[c] ^ 1;
    const double* Kp = Kbuf + (long)other * half + c * kk;
    const TB* Bpg = Bp + (long)c * dy * ldb;
    // B's staging, the states and the pivots' reciprocals share one barrier (the
    // reciprocals are used only where the proposal's factor exists)
    const TB* Bpc = stage_b(Bpg, dy, ldb, red + DU_RED, false);
    const int ldl = dual_ldl(ldb, sizeof(TB) == 2);  // row stride of Bpc
    for (int j = tid; j < r; j += TPB) {
        xs[j] = x[(long)c * r + j];
        ps[j] = xp[(long)c * r + j];
        ga[j] = gp[(long)c * r + j];
    }
    load_inv_diag(Kp, dy, invd, false);
    __syncthreads();
    const int okc = okp[c];
    if (state == CHAIN_FRESH) {
        if (tid == 0) {
            if (!okc) failures[c] += 1;
            phin = phip[c];
            phi[c] = phin;
            logdet[c] = logdetp[c];
            cur[c] = other;
            decision = 1;
            accflag[c] = 2;
        }
        __syncthreads();
    } else {
        double rev = 0.0;
        if (okc)
            rev = dual_rho0(Bpc, ldl, Kp, invd, r, dy, dt, s, beta, ps, xs, ga, logdetp[c], v, mh, t1, t2, z, acc,
                            red, dinv);
        if (tid == 0) {
            const double lr = phi[c] - phip[c] + rev - lfwd[c];
            const double u = philox_uniform(meta.key0[c], meta.key1[c], (uint64_t)step, (uint64_t)meta.index[c]);
            const bool good = okc && isfinite(lr);
            const bool accept = good && (log(u) <= lr);
            if (!good) failures[c] += 1;
            phin = phi[c];
            if (da) {
                // delayed acceptance: a pass goes to the second stage, which commits
                decision = 0;
                accflag[c] = accept ? 3 : 0;
            } else {
                decision = accept ? 1 : 0;
                if (accept) {
                    accepts[c] += 1;
                    phin = phip[c];
                    phi[c] = phin;
                    logdet[c] = logdetp[c];
                    cur[c] = other;
                }
                accflag[c] = decision;
            }
        }
    }
    __syncthreads();
    if (decision) {
        for (int j = tid; j < r; j += TPB) {
            x[(long)c * r + j] = ps[j];
            g[(long)c * r + j] = ga[j];
        }
        TB* Bsc = Bs + (long)c * dy * ldb;
        if constexpr (sizeof(TB) == 2) {
            // from the staged copy (row stride ldl), 16 bytes per move (ldb: a multiple of 32)
            const int c16 = ldb / 8, l16 = ldl / 8;
            const uint4* src = reinterpret_cast<const uint4*>(Bpc);
            uint4* dst = reinterpret_cast<uint4*>(Bsc);
            for (long e = tid; e < (long)dy * c16; e += TPB) dst[e] = src[(e / c16) * l16 + e % c16];
        } else {
            for (long e = tid; e < (long)dy * ldb; e += TPB) Bsc[e] = Bpg[e];
        }
    }
    if (!da) finish_chain(c, r, meta, state, step, decision ? ps : xs, phin, rec);
}

// log rho^(1) of the dual form at given states and caches (the stage entry point): the
// forward term with the cache of x, the reverse term with the cache of xp, both by
// dual_rho0 (the acceptance kernel's reverse-term code). K: n x dy x dy factors, B: n x dy x ldb.
template <typename TB>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(2, 2)))
void log_rho_dual_kernel(int r, int dy, int ldb, double dt, double s, double beta, const double* __restrict__ x,
                         const double* __restrict__ phi_x, const double* __restrict__ g_x, const TB* __restrict__ Bx,
                         const double* __restrict__ Kx, const double* __restrict__ logdet_x,
                         const double* __restrict__ xp, const double* __restrict__ phi_p,
                         const double* __restrict__ g_p, const TB* __restrict__ Bp, const double* __restrict__ Kp,
                         const double* __restrict__ logdet_p, double* __restrict__ out) {
    extern __shared__ double dyn[];
    double* R = dyn;
    double *xs = R, *ps = R + r, *ga = R + 2 * r, *v = R + 3 * r, *mh = R + 4 * r;
    double* Y = dyn + (size_t)DU_NR * r;
    double *invd = Y, *t1 = Y + dy, *t2 = Y + 2 * dy, *z = Y + 3 * dy;
    double* acc = Y + (size_t)DU_NY * dy;
    double* red = acc + 9 * SB;
    const int c = blockIdx.x, tid = threadIdx.x;
    const long kk = (long)dy * dy;
    const int ldl = dual_ldl(ldb, sizeof(TB) == 2);
    for (int j = tid; j < r; j += TPB) {
        xs[j] = x[(long)c * r + j];
        ps[j] = xp[(long)c * r + j];
        ga[j] = g_x[(long)c * r + j];
    }
    __syncthreads();
    const TB* B1 = stage_b(Bx + (long)c * dy * ldb, dy, ldb, red + DU_RED);
    load_inv_diag(Kx + c * kk, dy, invd);
    const double fwd = dual_rho0(B1, ldl, Kx + c * kk, invd, r, dy, dt, s, beta, xs, ps, ga, logdet_x[c], v, mh, t1,
                                 t2, z, acc, red, 0);
    __syncthreads();  // every thread is done with B1, invd and ga
    for (int j = tid; j < r; j += TPB) ga[j] = g_p[(long)c * r + j];
    __syncthreads();
    const TB* B2 = stage_b(Bp + (long)c * dy * ldb, dy, ldb, red + DU_RED);
    load_inv_diag(Kp + c * kk, dy, invd);
    const double rev = dual_rho0(B2, ldl, Kp + c * kk, invd, r, dy, dt, s, beta, ps, xs, ga, logdet_p[c], v, mh, t1,
                                 t2, z, acc, red, 0);
    if (tid == 0) out[c] = phi_x[c] - phi_p[c] + rev - fwd;
}

// ---------------------------------------------------------------------------------
// Delayed acceptance: the second stage of Alg. 1 (eq. da_dino_trr_2). The first-stage
// acceptance kernel marks a pass with accflag 3 and commits nothing; the passes are
// compacted into the first rows of a batch, the true-model stand-in runs on those rows
// only (its launches skip row tiles past the count), and the second-stage kernel
// decides, commits and ends every chain's step. The complement kernel then moves the
// complement of the committed chains with the draws the gather used.

// One wave per chain: a pass takes the next batch row and writes the coordinates the
// true model reads: x+ and the pCN move of the first rT - r complement coordinates (the
// complement kernel's draws and expression, so the true model sees the state a commit
// leaves). Chains that did not pass get pos -1.
__global__ __launch_bounds__(64) void da_gather_kernel(int r, int rT, int ldz, double s, double beta, ChainMeta meta,
                                                       const int32_t* __restrict__ accflag, const double* __restrict__ xp,
                                                       const float* __restrict__ z, int32_t* npass,
                                                       int32_t* __restrict__ pos, double* __restrict__ zin) {
    const int c = blockIdx.x, tid = threadIdx.x;
    __shared__ int slot;
    if (accflag[c] != 3) {
        if (tid == 0) pos[c] = -1;
        return;
    }
    if (tid == 0) {
        slot = atomicAdd(npass, 1);
        pos[c] = slot;
    }
    __syncthreads();
    double* row = zin + (long)slot * rT;
    for (int j = tid; j < r; j += 64) row[j] = xp[(long)c * r + j];
    const int extra = rT - r;
    if (extra > 0) {
        const float* zc = z + (long)c * ldz;
        const uint64_t k0 = meta.key0[c], k1 = meta.key1[c];
        const uint64_t step = (uint64_t)meta.step[c], chain = (uint64_t)meta.index[c];
        for (int b4 = tid; 4 * b4 < extra; b4 += 64) {
            double nv[4];
            philox_normals4(k0, k1, (uint64_t)b4, STREAM_COMPLEMENT, step, chain, nv);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 4 * b4 + q;
                if (k < extra) row[r + k] = (double)pcn_move(zc[k], nv[q], s, beta);
            }
        }
    }
}

// The true model's input rows at the states themselves (chain initialisation): row c of
// the batch is chain c; the batch holds all n chains.
__global__ __launch_bounds__(64) void da_init_kernel(int n, int r, int rT, int ldz, const double* __restrict__ x,
                                                     const float* __restrict__ z, int32_t* npass,
                                                     int32_t* __restrict__ pos, double* __restrict__ zin) {
    const int c = blockIdx.x, tid = threadIdx.x;
    if (tid == 0) {
        pos[c] = c;
        if (c == 0) *npass = n;
    }
    double* row = zin + (long)c * rT;
    for (int j = tid; j < r; j += 64) row[j] = x[(long)c * r + j];
    for (int k = tid; k < rT - r; k += 64) row[r + k] = (double)z[(long)c * ldz + k];
}

// Dense basis: a pass takes the next batch row and writes its whole unprojected
// complement draw w+ = pCN move of w (every one of the d_m coordinates; the complement
// kernel's draws and expression) and its chain. One block per chain.
template <typename TW>
__global__ __launch_bounds__(256) void da_gather_dense_kernel(int d_m, int ldz, double s, double beta, ChainMeta meta,
                                                              const int32_t* __restrict__ accflag,
                                                              const float* __restrict__ z, int32_t* npass,
                                                              int32_t* __restrict__ pos, int32_t* __restrict__ rowchain,
                                                              TW* __restrict__ wb, int ldw) {
    const int c = blockIdx.x, tid = threadIdx.x;
    __shared__ int slot;
    if (accflag[c] != 3) {
        if (tid == 0) pos[c] = -1;
        return;
    }
    if (tid == 0) {
        slot = atomicAdd(npass, 1);
        pos[c] = slot;
        rowchain[slot] = c;
    }
    __syncthreads();
    const float* zc = z + (long)c * ldz;
    TW* row = wb + (long)slot * ldw;
    const uint64_t k0 = meta.key0[c], k1 = meta.key1[c];
    const uint64_t step = (uint64_t)meta.step[c], chain = (uint64_t)meta.index[c];
    for (int b4 = tid; 4 * b4 < d_m; b4 += 256) {
        double nv[4];
        philox_normals4(k0, k1, (uint64_t)b4, STREAM_COMPLEMENT, step, chain, nv);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = 4 * b4 + q;
            if (k < d_m) row[k] = (TW)pcn_move(zc[k], nv[q], s, beta);
        }
    }
}

// Dense basis at initialisation: row c of the batch is chain c's own w.
template <typename TW>
__global__ __launch_bounds__(256) void da_init_dense_kernel(int n, int d_m, int ldz, const float* __restrict__ z,
                                                            int32_t* npass, int32_t* __restrict__ pos,
                                                            int32_t* __restrict__ rowchain, TW* __restrict__ wb,
                                                            int ldw) {
    const int c = blockIdx.x, tid = threadIdx.x;
    if (tid == 0) {
        pos[c] = c;
        rowchain[c] = c;
        if (c == 0) *npass = n;
    }
    for (int k = tid; k < d_m; k += 256) wb[(long)c * ldw + k] = (TW)z[(long)c * ldz + k];
}

// Alg. 1's assembly of the full parameter in whitened coordinates, the r_T coordinates the
// true model reads: zin[q][i] = w[q][i] + sum_j u_j[i] (x[c][j] - t[q][j]), with t = U^T w
// (the projection GEMM before this kernel), c = rowchain[q]; rows past the batch count
// return. One block per batch row.
template <typename TW, typename TT>
__global__ __launch_bounds__(256) void da_assemble_kernel(int r, int rT, int d_m, int ldw, const int32_t* npass,
                                                          const int32_t* __restrict__ rowchain,
                                                          const double* __restrict__ xsrc, const double* __restrict__ UT,
                                                          const TW* __restrict__ wb, const TT* __restrict__ tp,
                                                          double* __restrict__ zin) {
    const int q = blockIdx.x;
    if (q >= *npass) return;
    const int c = rowchain[q];
    __shared__ double a[512];
    for (int j = threadIdx.x; j < r; j += 256) a[j] = xsrc[(long)c * r + j] - (double)tp[(long)q * r + j];
    __syncthreads();
    for (int i = threadIdx.x; i < rT; i += 256) {
        double acc = (double)wb[(long)q * ldw + i];
        for (int j = 0; j < r; ++j) acc += UT[(long)j * d_m + i] * a[j];
        zin[(long)q * rT + i] = acc;
    }
}

// True misfit Phi = 1/2 |Gamma^-1/2 (y - f_T)|^2 of chain c from batch row pos[c] (pos
// null: row c); with npass_reset, the batch count is cleared for the next step.
template <typename TF>
__global__ __launch_bounds__(64) void true_misfit_kernel(int dy, ChainMeta meta, const TF* __restrict__ fT,
                                                         const int32_t* __restrict__ pos, const double* __restrict__ y,
                                                         const double* __restrict__ winv, double* __restrict__ out,
                                                         int32_t* npass_reset) {
    const int c = blockIdx.x, tid = threadIdx.x;
    const long pr = pos ? pos[c] : c;
    const long rq = meta.row ? meta.row[c] : 0;
    double a = 0.0;
    for (int i = tid; i < dy; i += 64) {
        const double e = (y[rq * dy + i] - (double)fT[pr * dy + i]) * winv[rq * dy + i];
        a += e * e;
    }
    a = wave_sum(a);
    if (tid == 0) {
        out[c] = 0.5 * a;
        if (c == 0 && npass_reset) *npass_reset = 0;
    }
}

// Second stage: for a pass, the true misfit at the full proposal (batch row pos[c]),
// log rho^(2) = (Phi~(x+) - Phi~(x)) + (Phi(m) - Phi(m+)) and the decision with the
// uniform of stream 5; a commit takes the proposal and its caches (factor half flip, the
// proposal's B in the dual form, the true misfit). Every chain's step ends here (trace
// row, running sums, step counter). accflag leaves 1 for committed moves (the complement
// kernel moves them) and 0 otherwise.
template <typename TB, typename TF>
__global__ __launch_bounds__(TPB) void da_accept_kernel(int r, int dy, long bcount, ChainMeta meta, double* x, double* g,
                                                        double* phi, double* logdet, int32_t* cur, const double* xp,
                                                        const double* gp, const double* phip, const double* logdetp,
                                                        const TF* __restrict__ fT, const double* __restrict__ y,
                                                        const double* __restrict__ winv, double* phit,
                                                        int32_t* accflag, const int32_t* __restrict__ pos,
                                                        int32_t* npass, int64_t* accepts, int64_t* failures,
                                                        int64_t* passes, const TB* __restrict__ Bp, TB* __restrict__ Bs,
                                                        StepRecord rec) {
    __shared__ int decision;
    __shared__ double red[TPB / 64];
    const int c = blockIdx.x, tid = threadIdx.x;
    if (c == 0 && tid == 0) *npass = 0;  // this step's batch has been evaluated
    const int32_t state = chain_state(meta, c);
    if (state == CHAIN_IDLE) {
        return;
    }
    const int64_t step = meta.step[c];  // read by every thread before the finish advances it
    const int flag = accflag[c];
    double phin = 0.0;
    if (flag == 3) {
        const long pr = pos[c];
        const long rq = meta.row ? meta.row[c] : 0;
        double a = 0.0;
        for (int i = tid; i < dy; i += TPB) {
            const double e = (y[rq * dy + i] - (double)fT[pr * dy + i]) * winv[rq * dy + i];
            a += e * e;
        }
        a = block_sum(a, red);
        if (tid == 0) {
            const double phitp = 0.5 * a;
            const double lr2 = (phip[c] - phi[c]) + (phit[c] - phitp);
            const double u2 = philox_uniform_stream(meta.key0[c], meta.key1[c], STREAM_UNIFORM2, (uint64_t)step,
                                                    (uint64_t)meta.index[c]);
            const bool good = isfinite(lr2);
            const bool accept = good && (log(u2) <= lr2);
            passes[c] += 1;
            if (!good) failures[c] += 1;
            phin = phi[c];
            if (accept) {
                accepts[c] += 1;
                phin = phip[c];
                phi[c] = phin;
                logdet[c] = logdetp[c];
                cur[c] ^= 1;
                phit[c] = phitp;
            }
            decision = accept ? 1 : 0;
            accflag[c] = decision;
        }
        __syncthreads();
        if (decision) {
            for (int j = tid; j < r; j += TPB) {
                x[(long)c * r + j] = xp[(long)c * r + j];
                g[(long)c * r + j] = gp[(long)c * r + j];
            }
            if (Bs)
                for (long e = tid; e < bcount; e += TPB) Bs[(long)c * bcount + e] = Bp[(long)c * bcount + e];
        }
    } else {
        // rejected in the first stage (or a fresh chain, committed there)
        if (tid == 0) {
            phin = phi[c];
            decision = flag == 2 ? 1 : 0;
        }
        __syncthreads();
    }
    finish_chain(c, r, meta, state, step, decision ? xp + (long)c * r : x + (long)c * r, phin, rec);
}

// Copies the Jacobian of every chain (n x dy x ldb values) into the state's buffer.
template <typename TB>
__global__ void copy_b_kernel(long count, const TB* __restrict__ src, TB* __restrict__ dst) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x)
        dst[e] = src[e];
}

// pCN move of the complement on accepted chains: z <- s z + beta zeta (FP32 state). Runs
// after the accept kernel of the same step.
// Grid: nbx blocks per chain, chain c = blockIdx.y; with FOLD (more chains than the
// grid's y extent) a 1-D grid, chain c = blockIdx.x / nbx.
template <bool FOLD>
__global__ __launch_bounds__(TPB) void complement_kernel(int nbx, int d_perp, int ldz, double s, double beta,
                                                         ChainMeta meta, const int32_t* __restrict__ accflag,
                                                         float* z) {
    const int c = FOLD ? (int)(blockIdx.x / nbx) : (int)blockIdx.y;
    const int flag = accflag[c];
    if (!flag) return;
    const int bx = FOLD ? (int)blockIdx.x - c * nbx : (int)blockIdx.x;
    const int b4 = bx * TPB + threadIdx.x;
    const int j0 = 4 * b4;
    if (j0 >= d_perp) return;
    double nv[4];
    float* zc = z + (long)c * ldz;
    if (flag == 2) {
        // a fresh chain: the complement starts from a prior draw (stream 4)
        philox_normals4(meta.key0[c], meta.key1[c], (uint64_t)b4, STREAM_INIT_Z, 0, (uint64_t)meta.index[c], nv);
        for (int q = 0; q < 4 && j0 + q < d_perp; ++q) zc[j0 + q] = (float)nv[q];
        return;
    }
    // the accept kernel has already advanced the step counter of this (live) chain
    philox_normals4(meta.key0[c], meta.key1[c], (uint64_t)b4, STREAM_COMPLEMENT, (uint64_t)(meta.step[c] - 1),
                    (uint64_t)meta.index[c], nv);
    if (j0 + 3 < d_perp) {
        float4 v = *reinterpret_cast<const float4*>(zc + j0);
        v.x = pcn_move(v.x, nv[0], s, beta);
        v.y = pcn_move(v.y, nv[1], s, beta);
        v.z = pcn_move(v.z, nv[2], s, beta);
        v.w = pcn_move(v.w, nv[3], s, beta);
        *reinterpret_cast<float4*>(zc + j0) = v;
    } else {
        for (int q = 0; q < 4 && j0 + q < d_perp; ++q) zc[j0 + q] = pcn_move(zc[j0 + q], nv[q], s, beta);
    }
}

__global__ void meta_fill_kernel(ChainMeta meta, double* __restrict__ sumx, int r, int c0, int n, uint64_t key0,
                                 uint64_t key1, int64_t budget, int64_t burn, int32_t row, int32_t state,
                                 int32_t first_index) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const int c = c0 + k;
        meta.key0[c] = key0;
        meta.key1[c] = key1;
        meta.step[c] = 0;
        meta.budget[c] = budget;
        meta.burn[c] = burn;
        meta.index[c] = first_index + k;
        meta.row[c] = row;
        meta.state[c] = state;
        if (sumx)
            for (int j = 0; j < r; ++j) sumx[(long)c * r + j] = 0.0;
    }
}

// xbar_j = sum over chains [c0, c0 + n) of sumx_cj / (n count); one block.
__global__ __launch_bounds__(256) void request_xbar_kernel(int r, int c0, int n, double inv,
                                                           const double* __restrict__ sumx,
                                                           double* __restrict__ xbar) {
    for (int j = threadIdx.x; j < r; j += 256) {
        double acc = 0.0;
        for (int c = c0; c < c0 + n; ++c) acc += sumx[(long)c * r + j];
        xbar[j] = acc * inv;
    }
}

// field_p = sum_k Psi[p][k] xbar_k: one wave per node row of the basis (d_m x r).
__global__ __launch_bounds__(256) void decode_kernel(int d_m, int r, const double* __restrict__ dec,
                                                     const double* __restrict__ xbar, double* __restrict__ field) {
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= d_m) return;
    double acc = 0.0;
    for (int k = lane; k < r; k += 64) acc += dec[(long)p * r + k] * xbar[k];
    acc = wave_sum(acc);
    if (lane == 0) field[p] = acc;
}

// Normals of one stream for n chains at one step: out[c][k], k < count.
__global__ void normals_kernel(uint64_t seed, uint64_t rid, int n, int stream_id, int64_t step, int count,
                               double* out, long ldo, int as_float, float* outf) {
    const int b4 = blockIdx.x * blockDim.x + threadIdx.x;
    if (4 * b4 >= count) return;
    for (int c = blockIdx.y; c < n; c += gridDim.y) {  // the grid's y extent is capped at GRID_Y_MAX
        double nv[4];
        philox_normals4(seed, rid, (uint64_t)b4, (uint64_t)stream_id, (uint64_t)step, (uint64_t)c, nv);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = 4 * b4 + q;
            if (k < count) {
                if (as_float) outf[(long)c * ldo + k] = (float)nv[q];
                else out[(long)c * ldo + k] = nv[q];
            }
        }
    }
}

__global__ void copy_rows_kernel(int n, int width, const double* __restrict__ src, double* __restrict__ dst) {
    const long total = (long)n * width;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x)
        dst[e] = src[e];
}

// ---------------------------------------------------------------------------------
static size_t chol_lds(int r) { return (size_t)r * CLDP * sizeof(double); }
static size_t panel_lds(int r) { return ((size_t)PNB * (r | 1) + PNB) * sizeof(double); }
static int ldz_of(int d_perp) { return (d_perp + 63) / 64 * 64; }

// Factor kernels by variant: 0-2 one wavefront per chain (orders up to 32, 56, 104), 3-4
// a 512-thread block per chain with the triangle in registers (up to 128, 208), 5 the
// LDS panel kernel (up to 512), 6 the transposed-panel kernel with a one-wave diagonal
// block (up to 512). Any variant whose maximum covers the order is correct.
static const int kCholMax[CHOL_VARIANTS] = {32, 56, 104, 128, 208, 512, 512};

int cholesky_variant_max(int variant) { return (variant >= 0 && variant < CHOL_VARIANTS) ? kCholMax[variant] : 0; }

// The choice without a tuning entry: the smallest register or wavefront variant that holds
// the order, and above those the transposed-panel kernel (faster than the LDS panel kernel
// at every order it was timed at, 300 and 400).
static int default_cholesky_variant(int r) {
    for (int v = 0; v < 5; ++v)
        if (r <= kCholMax[v]) return v;
    return 6;
}

void launch_cholesky_variant(int variant, int n, int r, double* A, long strideA, const int32_t* slot, int slot_xor,
                             long slot_stride, double* logdet, int32_t* ok, hipStream_t st) {
    DINO_REQUIRE(variant >= 0 && variant < CHOL_VARIANTS && r <= kCholMax[variant], DINO_EINVAL,
                 "factor kernel variant does not hold this order");
    static bool attr_set = false;
    if (!attr_set) {
        DINO_HIP(hipFuncSetAttribute((const void*)cholesky_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     160 * 1024 - 256));
        DINO_HIP(hipFuncSetAttribute((const void*)cholesky_panel_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 256));
        attr_set = true;
    }
    switch (variant) {
    case 0:
        hipLaunchKernelGGL((cholesky_wave_kernel<4>), dim3(n), dim3(64), 0, st, r, A, strideA, slot, slot_xor,
                           slot_stride, logdet, ok);
        break;
    case 1:
        hipLaunchKernelGGL((cholesky_wave_kernel<7>), dim3(n), dim3(64), 0, st, r, A, strideA, slot, slot_xor,
                           slot_stride, logdet, ok);
        break;
    case 2:
        hipLaunchKernelGGL((cholesky_wave_kernel<13>), dim3(n), dim3(64), 0, st, r, A, strideA, slot, slot_xor,
                           slot_stride, logdet, ok);
        break;
    case 3:
        hipLaunchKernelGGL((cholesky_reg_kernel<512, 8, 4>), dim3(n), dim3(512), 0, st, r, A, strideA, slot,
                           slot_xor, slot_stride, logdet, ok);
        break;
    case 4:
        hipLaunchKernelGGL((cholesky_reg_kernel<512, 13, 7>), dim3(n), dim3(512), 0, st, r, A, strideA, slot,
                           slot_xor, slot_stride, logdet, ok);
        break;
    case 5:
        hipLaunchKernelGGL(cholesky_kernel, dim3(n), dim3(TPB), chol_lds(r), st, r, A, strideA, slot, slot_xor,
                           slot_stride, logdet, ok);
        break;
    default:
        hipLaunchKernelGGL(cholesky_panel_kernel, dim3(n), dim3(PTPB), panel_lds(r), st, r, A, strideA, slot,
                           slot_xor, slot_stride, logdet, ok);
        break;
    }
    DINO_HIP(hipGetLastError());
}

void launch_cholesky_slot(int n, int r, double* A, long strideA, const int32_t* slot, int slot_xor,
                          long slot_stride, double* logdet, int32_t* ok, hipStream_t st) {
    int v = tuned_choice(TUNE_CHOL, n, r, 0);
    if (v < 0 || cholesky_variant_max(v) < r) v = default_cholesky_variant(r);
    launch_cholesky_variant(v, n, r, A, strideA, slot, slot_xor, slot_stride, logdet, ok, st);
}

// Identity matrices of order r in the slot-selected halves (factor timing input).
__global__ void fill_identity_kernel(int r, double* A, long strideA, const int32_t* slot, int slot_xor,
                                     long slot_stride) {
    const int c = blockIdx.y;
    double* a = A + (long)c * strideA + slot_offset(slot, slot_xor, slot_stride, c);
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)r * r; e += (long)gridDim.x * blockDim.x)
        a[e] = (e / r == e % r) ? 1.0 : 0.0;
}

void launch_fill_identity(int n, int r, double* A, long strideA, const int32_t* slot, int slot_xor, long slot_stride,
                          hipStream_t st) {
    const int bx = (int)std::min<long>(((long)r * r + 255) / 256, 64);
    for (int c0 = 0; c0 < n; c0 += (int)GRID_Y_MAX) {
        const int cn = std::min(n - c0, (int)GRID_Y_MAX);
        hipLaunchKernelGGL(fill_identity_kernel, dim3(bx, cn), dim3(256), 0, st, r, A + (long)c0 * strideA, strideA,
                           slot ? slot + c0 : nullptr, slot_xor, slot_stride);
    }
    DINO_HIP(hipGetLastError());
}


// LDS of the transition kernels (r vectors, solve scratch and product partial sums).
constexpr size_t CH_LDS_LIMIT = 160 * 1024 - 1024;
static size_t chain_lds_bytes(int r) { return chain_lds_doubles(r) * sizeof(double); }

bool dual_lds_fits(int r, int dy, bool bf16) {
    const int ldb = bf16 ? (r + 31) / 32 * 32 : r;
    return dual_lds_doubles(r, dy, ldb, bf16) * sizeof(double) <= CH_LDS_LIMIT;
}

template <typename K>
static void allow_large_lds(K kernel, bool& done) {
    if (!done) {
        DINO_HIP(hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)CH_LDS_LIMIT));
        done = true;
    }
}

void launch_propose_slot(dino_problem* p, int n, const double* x, const double* g, const double* L, long strideL,
                         const int32_t* slot, int slot_xor, long slot_stride, const double* xi_given, bool use_meta,
                         double* xp, double* lfwd, const double* logdet, hipStream_t st) {
    static bool attr = false;
    allow_large_lds(propose_kernel, attr);
    const ChainMeta meta = use_meta ? p->meta : ChainMeta{};
    hipLaunchKernelGGL(propose_kernel, dim3(n), dim3(TPB), chain_lds_bytes(p->r), st, p->r, p->s, p->beta, meta, x,
                       g, L, strideL, slot, slot_xor, slot_stride, xi_given, logdet, xp, lfwd);
    DINO_HIP(hipGetLastError());
}


// The step record of a problem's transitions (trace rows by the chains' step counters).
static StepRecord step_record(dino_problem* p) {
    return StepRecord{p->sumx, p->xtrace, p->phitrace, p->xtrace ? (int64_t)p->desc.trace_capacity : 0, p->C};
}

void launch_accept(dino_problem* p, int n, hipStream_t st) {
    static bool attr = false;
    allow_large_lds(accept_kernel, attr);
    const long half = (long)p->C * p->r * p->r;
    hipLaunchKernelGGL(accept_kernel, dim3(n), dim3(TPB), chain_lds_bytes(p->r), st, p->r, p->desc.dt, p->s, p->beta,
                       p->meta, p->x, p->g, p->phi, p->logdet, p->Lbuf, half, p->cur, p->xp, p->gp, p->phip,
                       p->logdetp, p->okp, p->lfwd, p->accepts, p->failures, p->acc, step_record(p),
                       p->da ? 1 : 0);
    DINO_HIP(hipGetLastError());
}

void launch_pcn_propose(dino_problem* p, int n, hipStream_t st) {
    hipLaunchKernelGGL(pcn_propose_kernel, dim3(n), dim3(64), 0, st, p->r, p->s, p->beta, p->meta, p->x, p->xp);
    DINO_HIP(hipGetLastError());
}

// The forward stage leaves the network output in p->f (FP64 path) or p->f32 (BF16 path).
void launch_pcn_accept(dino_problem* p, int n, hipStream_t st) {
    const StepRecord rec = step_record(p);
    const double* lterm = p->desc.method == DINO_METHOD_LAPCN ? p->lfwd : nullptr;
    if (p->desc.precision == DINO_PREC_F64)
        hipLaunchKernelGGL(pcn_accept_kernel<double>, dim3(n), dim3(TPB), 0, st, p->r, p->d_y, p->meta, p->f, p->y,
                           p->winv, p->x, p->phi, p->xp, lterm, p->accepts, p->failures, p->acc, rec);
    else
        hipLaunchKernelGGL(pcn_accept_kernel<float>, dim3(n), dim3(TPB), 0, st, p->r, p->d_y, p->meta, p->f32, p->y,
                           p->winv, p->x, p->phi, p->xp, lterm, p->accepts, p->failures, p->acc, rec);
    DINO_HIP(hipGetLastError());
}

void launch_lapcn_propose(dino_problem* p, int n, hipStream_t st) {
    static bool attr = false;
    allow_large_lds(lapcn_propose_kernel, attr);
    hipLaunchKernelGGL(lapcn_propose_kernel, dim3(n), dim3(TPB), chain_lds_bytes(p->r), st, p->r, p->s, p->beta,
                       p->meta, p->x, p->Lfix, p->xmap, p->xp, p->lfwd);
    DINO_HIP(hipGetLastError());
}

// The fixed diagonal metric of a DIS-mMALA problem (null for MALA).
static const double* dis_metric(const dino_problem* p) {
    return p->desc.method == DINO_METHOD_DIS_MMALA ? p->ctx->basis.lam_dis : nullptr;
}

void launch_mala_propose(dino_problem* p, int n, hipStream_t st) {
    hipLaunchKernelGGL(mala_propose_kernel, dim3(n), dim3(64), 0, st, p->r, p->desc.dt, p->s, p->beta, p->meta, p->x,
                       p->g, p->xp, p->lfwd, dis_metric(p));
    DINO_HIP(hipGetLastError());
}

void launch_mala_accept(dino_problem* p, int n, hipStream_t st) {
    hipLaunchKernelGGL(mala_accept_kernel, dim3(n), dim3(TPB), 0, st, p->r, p->desc.dt, p->s, p->beta, p->meta, p->x,
                       p->g, p->phi, p->xp, p->gp, p->phip, p->lfwd, p->accepts, p->failures, p->acc,
                       step_record(p), dis_metric(p));
    DINO_HIP(hipGetLastError());
}

void launch_log_rho(dino_problem* p, int n, const double* x, const double* phi_x, const double* g_x,
                    const double* L_x, const double* logdet_x, const double* xp, const double* phi_p,
                    const double* g_p, const double* L_p, const double* logdet_p, double* out, hipStream_t st) {
    static bool attr = false;
    allow_large_lds(log_rho_kernel, attr);
    hipLaunchKernelGGL(log_rho_kernel, dim3(n), dim3(TPB), chain_lds_bytes(p->r), st, p->r, p->desc.dt, p->s,
                       p->beta, x, phi_x, g_x, L_x, logdet_x, xp, phi_p, g_p, L_p, logdet_p, out);
    DINO_HIP(hipGetLastError());
}

// The dual kernels of a step solve with the inverted diagonal blocks where the problem's
// factors carry them (the fused Gram + factor kernel writes them) and the tuning entry
// (d_y) does not ask for the substitution sweeps.
static bool dual_solve_dinv(const dino_problem* p) {
    return p->dinv && tuned_choice(TUNE_DUALSOLVE, p->d_y, 0, 0) != 0;
}

template <typename TB>
static void propose_dual_t(dino_problem* p, int n, const TB* Bs, int ldb, hipStream_t st) {
    static bool attr = false;
    allow_large_lds(propose_dual_kernel<TB>, attr);
    const long kk = (long)p->d_y * p->d_y;
    const bool bf = sizeof(TB) == 2;
    hipLaunchKernelGGL(propose_dual_kernel<TB>, dim3(n), dim3(TPB),
                       dual_lds_doubles(p->r, p->d_y, ldb, bf) * sizeof(double),
                       st, p->r, p->d_y, ldb, p->desc.dt, p->s, p->beta, p->meta, p->x, p->g, Bs, p->Lbuf, kk,
                       p->cur, 0, (long)p->C * kk, p->logdet, (const double*)nullptr, p->xp, p->lfwd,
                       dual_solve_dinv(p) ? 1 : 0);
    DINO_HIP(hipGetLastError());
}

// Stage entry points of the dual form on caller buffers: every chain is live, the
// normals are given, the factors are packed n x dy x dy.
template <typename TB>
static void eval_propose_dual_t(dino_problem* p, int n, const double* x, const double* g, const TB* B, int ldb,
                                const double* K, const double* logdet, const double* xi, double* xp, double* lfwd,
                                hipStream_t st) {
    static bool attr = false;
    allow_large_lds(propose_dual_kernel<TB>, attr);
    const long kk = (long)p->d_y * p->d_y;
    hipLaunchKernelGGL(propose_dual_kernel<TB>, dim3(n), dim3(TPB),
                       dual_lds_doubles(p->r, p->d_y, ldb, sizeof(TB) == 2) * sizeof(double), st, p->r, p->d_y, ldb,
                       p->desc.dt, p->s, p->beta, ChainMeta{}, x, g, B, K, kk, (const int32_t*)nullptr, 0, 0L, logdet,
                       xi, xp, lfwd, 0);
    DINO_HIP(hipGetLastError());
}

template <typename TB>
static void eval_log_rho_dual_t(dino_problem* p, int n, int ldb, const double* x, const double* phi_x,
                                const double* g_x, const TB* B_x, const double* K_x, const double* logdet_x,
                                const double* xp, const double* phi_p, const double* g_p, const TB* B_p,
                                const double* K_p, const double* logdet_p, double* out, hipStream_t st) {
    static bool attr = false;
    allow_large_lds(log_rho_dual_kernel<TB>, attr);
    hipLaunchKernelGGL(log_rho_dual_kernel<TB>, dim3(n), dim3(TPB),
                       dual_lds_doubles(p->r, p->d_y, ldb, sizeof(TB) == 2) * sizeof(double), st, p->r, p->d_y, ldb,
                       p->desc.dt, p->s, p->beta, x, phi_x, g_x, B_x, K_x, logdet_x, xp, phi_p, g_p, B_p, K_p,
                       logdet_p, out);
    DINO_HIP(hipGetLastError());
}

int jacobian_ld(const dino_problem* p) {
    return p->desc.precision == DINO_PREC_F64 ? p->r : (p->r + 31) / 32 * 32;
}

void launch_eval_propose_dual(dino_problem* p, int n, const double* x, const double* g, const void* B,
                              const double* K, const double* logdet, const double* xi, double* xp, double* lfwd,
                              hipStream_t st) {
    const int ldb = jacobian_ld(p);
    if (p->desc.precision == DINO_PREC_F64)
        eval_propose_dual_t<double>(p, n, x, g, (const double*)B, ldb, K, logdet, xi, xp, lfwd, st);
    else
        eval_propose_dual_t<__hip_bfloat16>(p, n, x, g, (const __hip_bfloat16*)B, ldb, K, logdet, xi, xp, lfwd, st);
}

void launch_eval_log_rho_dual(dino_problem* p, int n, const double* x, const double* phi_x, const double* g_x,
                              const void* B_x, const double* K_x, const double* logdet_x, const double* xp,
                              const double* phi_p, const double* g_p, const void* B_p, const double* K_p,
                              const double* logdet_p, double* out, hipStream_t st) {
    const int ldb = jacobian_ld(p);
    if (p->desc.precision == DINO_PREC_F64)
        eval_log_rho_dual_t<double>(p, n, ldb, x, phi_x, g_x, (const double*)B_x, K_x, logdet_x, xp, phi_p, g_p,
                                    (const double*)B_p, K_p, logdet_p, out, st);
    else
        eval_log_rho_dual_t<__hip_bfloat16>(p, n, ldb, x, phi_x, g_x, (const __hip_bfloat16*)B_x, K_x, logdet_x, xp,
                                            phi_p, g_p, (const __hip_bfloat16*)B_p, K_p, logdet_p, out, st);
}

// The stored Jacobian of chains [0, n) as FP64 rows of r values (n x dy x r).
template <typename TB>
__global__ void jacobian_to_double_kernel(long total, int r, int ldb, const TB* __restrict__ B, double* __restrict__ out) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const long row = e / r;
        const int j = (int)(e - row * r);
        out[e] = to_d(B[row * ldb + j]);
    }
}

void launch_jacobian_to_double(dino_problem* p, int n, double* out, hipStream_t st) {
    const long total = (long)n * p->d_y * p->r;
    const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
    if (p->desc.precision == DINO_PREC_F64)
        hipLaunchKernelGGL(jacobian_to_double_kernel<double>, dim3(blocks), dim3(256), 0, st, total, p->r, p->r,
                           (const double*)p->Bj, out);
    else
        hipLaunchKernelGGL(jacobian_to_double_kernel<__hip_bfloat16>, dim3(blocks), dim3(256), 0, st, total, p->r,
                           jacobian_ld(p), (const __hip_bfloat16*)p->B16, out);
    DINO_HIP(hipGetLastError());
}

template <typename TB>
static void accept_dual_t(dino_problem* p, int n, const TB* Bp, TB* Bs, int ldb, hipStream_t st) {
    static bool attr = false;
    allow_large_lds(accept_dual_kernel<TB>, attr);
    const long half = (long)p->C * p->d_y * p->d_y;
    const bool bf = sizeof(TB) == 2;
    hipLaunchKernelGGL(accept_dual_kernel<TB>, dim3(n), dim3(TPB),
                       dual_lds_doubles(p->r, p->d_y, ldb, bf) * sizeof(double),
                       st, p->r, p->d_y, ldb, p->desc.dt, p->s, p->beta, p->meta, p->x, p->g, p->phi, p->logdet,
                       p->Lbuf, half, p->cur, p->xp, p->gp, p->phip, p->logdetp, p->okp, p->lfwd, Bp, Bs,
                       p->accepts, p->failures, p->acc, step_record(p), p->da ? 1 : 0, dual_solve_dinv(p) ? 1 : 0);
    DINO_HIP(hipGetLastError());
}

void launch_propose_dual(dino_problem* p, int n, hipStream_t st) {
    if (p->desc.precision == DINO_PREC_F64) propose_dual_t<double>(p, n, p->Bs64, p->r, st);
    else propose_dual_t<__hip_bfloat16>(p, n, p->Bs16, (p->r + 31) / 32 * 32, st);
}

void launch_accept_dual(dino_problem* p, int n, hipStream_t st) {
    if (p->desc.precision == DINO_PREC_F64) accept_dual_t<double>(p, n, p->Bj, p->Bs64, p->r, st);
    else accept_dual_t<__hip_bfloat16>(p, n, p->B16, p->Bs16, (p->r + 31) / 32 * 32, st);
}

// Dense basis: the projection t = U^T w of the batch rows (a GEMM over d_m, FP64 on the FP64
// path, FP32 MFMA on the mixed path; row tiles past the count skip) and the assembly of the
// coordinates the true model reads, from the reduced states xsrc.
static void da_project_dense(dino_problem* p, int n, const double* xsrc, hipStream_t st) {
    const Basis& b = p->ctx->basis;
    if (p->desc.precision == DINO_PREC_F64) {
        launch_gemm_nt64(n, p->d_m, p->r, p->wb64, p->d_m, b.UT, p->tp64, p->r, p->npass, st);
        hipLaunchKernelGGL((da_assemble_kernel<double, double>), dim3(n), dim3(256), 0, st, p->r, p->rT, p->d_m,
                           p->d_m, p->npass, p->rowchain, xsrc, b.UT, p->wb64, p->tp64, p->zin);
    } else {
        const int ldw = ldz_of(p->d_perp);
        launch_gemm_nt32(n, p->d_m, p->r, p->wb32, ldw, b.UT32, p->tp32, p->r, p->npass, st);
        hipLaunchKernelGGL((da_assemble_kernel<float, float>), dim3(n), dim3(256), 0, st, p->r, p->rT, p->d_m, ldw,
                           p->npass, p->rowchain, xsrc, b.UT, p->wb32, p->tp32, p->zin);
    }
    DINO_HIP(hipGetLastError());
}

void launch_da_gather(dino_problem* p, int n, hipStream_t st) {
    if (p->ctx->basis.dense) {
        const int ldz = ldz_of(p->d_perp);
        if (p->desc.precision == DINO_PREC_F64)
            hipLaunchKernelGGL(da_gather_dense_kernel<double>, dim3(n), dim3(256), 0, st, p->d_m, ldz, p->s, p->beta,
                               p->meta, p->acc, p->z, p->npass, p->pos, p->rowchain, p->wb64, p->d_m);
        else
            hipLaunchKernelGGL(da_gather_dense_kernel<float>, dim3(n), dim3(256), 0, st, p->d_m, ldz, p->s, p->beta,
                               p->meta, p->acc, p->z, p->npass, p->pos, p->rowchain, p->wb32, ldz);
        DINO_HIP(hipGetLastError());
        da_project_dense(p, n, p->xp, st);
        return;
    }
    hipLaunchKernelGGL(da_gather_kernel, dim3(n), dim3(64), 0, st, p->r, p->rT, p->z ? ldz_of(p->d_perp) : 0, p->s,
                       p->beta, p->meta, p->acc, p->xp, p->z, p->npass, p->pos, p->zin);
    DINO_HIP(hipGetLastError());
}

void launch_true_misfit(dino_problem* p, int n, double* out, hipStream_t st) {
    if (p->desc.precision == DINO_PREC_F64)
        hipLaunchKernelGGL(true_misfit_kernel<double>, dim3(n), dim3(64), 0, st, p->d_y, p->meta, p->fT64,
                           (const int32_t*)nullptr, p->y, p->winv, out, (int32_t*)nullptr);
    else
        hipLaunchKernelGGL(true_misfit_kernel<float>, dim3(n), dim3(64), 0, st, p->d_y, p->meta, p->fT32,
                           (const int32_t*)nullptr, p->y, p->winv, out, (int32_t*)nullptr);
    DINO_HIP(hipGetLastError());
}

// The true misfit of the states of chains [0, n) (initialisation).
void launch_da_init(dino_problem* p, int n, hipStream_t st) {
    if (p->ctx->basis.dense) {
        const int ldz = ldz_of(p->d_perp);
        if (p->desc.precision == DINO_PREC_F64)
            hipLaunchKernelGGL(da_init_dense_kernel<double>, dim3(n), dim3(256), 0, st, n, p->d_m, ldz, p->z, p->npass,
                               p->pos, p->rowchain, p->wb64, p->d_m);
        else
            hipLaunchKernelGGL(da_init_dense_kernel<float>, dim3(n), dim3(256), 0, st, n, p->d_m, ldz, p->z, p->npass,
                               p->pos, p->rowchain, p->wb32, ldz);
        DINO_HIP(hipGetLastError());
        da_project_dense(p, n, p->x, st);
    } else {
        hipLaunchKernelGGL(da_init_kernel, dim3(n), dim3(64), 0, st, n, p->r, p->rT, p->z ? ldz_of(p->d_perp) : 0,
                           p->x, p->z, p->npass, p->pos, p->zin);
    }
    launch_true_forward(p, n, p->zin, p->npass, st);
    if (p->desc.precision == DINO_PREC_F64)
        hipLaunchKernelGGL(true_misfit_kernel<double>, dim3(n), dim3(64), 0, st, p->d_y, p->meta, p->fT64, p->pos, p->y,
                           p->winv, p->phit, p->npass);
    else
        hipLaunchKernelGGL(true_misfit_kernel<float>, dim3(n), dim3(64), 0, st, p->d_y, p->meta, p->fT32, p->pos, p->y,
                           p->winv, p->phit, p->npass);
    DINO_HIP(hipGetLastError());
}

void launch_da_accept(dino_problem* p, int n, hipStream_t st) {
    const StepRecord rec = step_record(p);
    if (p->desc.precision == DINO_PREC_F64) {
        const long bc = (long)p->d_y * p->r;
        hipLaunchKernelGGL((da_accept_kernel<double, double>), dim3(n), dim3(TPB), 0, st, p->r, p->d_y, bc, p->meta,
                           p->x, p->g, p->phi, p->logdet, p->cur, p->xp, p->gp, p->phip, p->logdetp, p->fT64, p->y,
                           p->winv, p->phit, p->acc, p->pos, p->npass, p->accepts, p->failures, p->passes,
                           (const double*)(p->dual ? p->Bj : nullptr), p->dual ? p->Bs64 : nullptr, rec);
    } else {
        const long bc = (long)p->d_y * jacobian_ld(p);
        hipLaunchKernelGGL((da_accept_kernel<__hip_bfloat16, float>), dim3(n), dim3(TPB), 0, st, p->r, p->d_y, bc,
                           p->meta, p->x, p->g, p->phi, p->logdet, p->cur, p->xp, p->gp, p->phip, p->logdetp, p->fT32,
                           p->y, p->winv, p->phit, p->acc, p->pos, p->npass, p->accepts, p->failures, p->passes,
                           (const __hip_bfloat16*)(p->dual ? p->B16 : nullptr), p->dual ? p->Bs16 : nullptr, rec);
    }
    DINO_HIP(hipGetLastError());
}

void launch_keep_jacobian(dino_problem* p, int n, hipStream_t st) {
    if (p->desc.precision == DINO_PREC_F64) {
        const long count = (long)n * p->d_y * p->r;
        hipLaunchKernelGGL(copy_b_kernel<double>, dim3((int)std::min<long>((count + 255) / 256, 8192)), dim3(256), 0,
                           st, count, (const double*)p->Bj, p->Bs64);
    } else {
        const long count = (long)n * p->d_y * ((p->r + 31) / 32 * 32);
        hipLaunchKernelGGL(copy_b_kernel<__hip_bfloat16>, dim3((int)std::min<long>((count + 255) / 256, 8192)),
                           dim3(256), 0, st, count, (const __hip_bfloat16*)p->B16, p->Bs16);
    }
    DINO_HIP(hipGetLastError());
}

void launch_complement(dino_problem* p, int n, hipStream_t st) {
    if (!p->z || p->d_perp == 0) return;
    const int nb4 = (p->d_perp + 3) / 4;
    const int nbx = (nb4 + TPB - 1) / TPB;
    if (n <= (int)GRID_Y_MAX)
        hipLaunchKernelGGL(complement_kernel<false>, dim3(nbx, n), dim3(TPB), 0, st, nbx, p->d_perp, ldz_of(p->d_perp),
                           p->s, p->beta, p->meta, p->acc, p->z);
    else
        hipLaunchKernelGGL(complement_kernel<true>, dim3((unsigned)((long)nbx * n)), dim3(TPB), 0, st, nbx,
                           p->d_perp, ldz_of(p->d_perp), p->s, p->beta, p->meta, p->acc, p->z);
    DINO_HIP(hipGetLastError());
}


void launch_meta_fill(dino_problem* p, int c0, int n, uint64_t key0, uint64_t key1, int64_t budget, int64_t burn,
                      int32_t row, int32_t state, int32_t first_index, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(meta_fill_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p->meta, p->sumx, p->r, c0, n,
                       key0, key1, budget, burn, row, state, first_index);
    DINO_HIP(hipGetLastError());
}

void launch_request_mean(dino_problem* p, int c0, int n, int64_t count, double* xbar, double* field,
                         hipStream_t st) {
    const double inv = 1.0 / ((double)n * (double)std::max<int64_t>(count, 1));
    hipLaunchKernelGGL(request_xbar_kernel, dim3(1), dim3(256), 0, st, p->r, c0, n, inv, p->sumx, xbar);
    const int d_m = p->ctx->basis.d_m;
    hipLaunchKernelGGL(decode_kernel, dim3((d_m + 3) / 4), dim3(256), 0, st, d_m, p->r, p->ctx->basis.dec, xbar,
                       field);
    DINO_HIP(hipGetLastError());
}

void launch_init_draws(dino_problem* p, int draw_x, int draw_z, hipStream_t st) {
    if (draw_x) {
        dim3 grid(((p->r + 3) / 4 + 255) / 256, grid_y(p->C));
        hipLaunchKernelGGL(normals_kernel, grid, dim3(256), 0, st, p->desc.seed, p->desc.request_id, p->C,
                           (int)STREAM_INIT_X, (int64_t)0, p->r, p->x, (long)p->r, 0, (float*)nullptr);
    }
    if (draw_z && p->z) {
        dim3 grid(((p->d_perp + 3) / 4 + 255) / 256, grid_y(p->C));
        hipLaunchKernelGGL(normals_kernel, grid, dim3(256), 0, st, p->desc.seed, p->desc.request_id, p->C,
                           (int)STREAM_INIT_Z, (int64_t)0, p->d_perp, (double*)nullptr, (long)ldz_of(p->d_perp),
                           1, p->z);
    }
    DINO_HIP(hipGetLastError());
}

void launch_normals(uint64_t seed, uint64_t rid, int n, int stream_id, int64_t step, int count, double* out,
                    hipStream_t st) {
    dim3 grid(((count + 3) / 4 + 255) / 256, grid_y(n));
    hipLaunchKernelGGL(normals_kernel, grid, dim3(256), 0, st, seed, rid, n, stream_id, step, count, out,
                       (long)count, 0, (float*)nullptr);
    DINO_HIP(hipGetLastError());
}

void launch_copy_rows(int n, int width, const double* src, double* dst, hipStream_t st) {
    const long total = (long)n * width;
    const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(copy_rows_kernel, dim3(blocks), dim3(256), 0, st, n, width, src, dst);
    DINO_HIP(hipGetLastError());
}

}  // namespace dino
