// Single-wave Cholesky step of a small SPD matrix held in registers (shared by the
// per-chain factor kernel and the fused Gram + factor kernel of the mixed path).
// Lane (g, q) = (lane / 8, lane % 8) of the wave holds rows g + 8m and columns q + 8c of
// the lower triangle (block pairs c <= m); col (8 MB doubles of LDS) carries the current
// column, pivs (8 MB doubles) the pivots. Synchronisation: __syncthreads() in a block of
// one wave, or (WS) a wavefront-scope fence where the wave runs alone in a larger block
// (LDS operations of one wave complete in order; the fence keeps the compiler from moving
// them across the step boundary).
#pragma once
#include <hip/hip_runtime.h>

namespace dino {

template <bool WS>
__device__ __forceinline__ void chol_sync() {
    if constexpr (WS) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    } else {
        __syncthreads();
    }
}

// Column j = 8 PH + JJ of the single-wave factorisation. The phase PH is a compile-time
// constant, so that every register index is one; within a phase only JJ changes, and
// it runs as a loop (the unrolled form of all columns was ~100 KB of code). LAST marks
// JJ = 7, where column j + 1 lies in the next register block. Column j was published
// to col by the previous step (or before the first). The step updates the column block
// of column j + 1 first, takes the next pivot from its lane (v_readlane) and publishes
// column j + 1 before the rest of the trailing update, so that the next step's LDS reads
// overlap that update and its pivot arithmetic waits for no LDS round trip.
// the double of lane `lane` (wave-uniform) in every lane
__device__ __forceinline__ double lane_value(double x, int lane) {
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <int MB, int PH, bool LAST, bool WS = false>
__device__ __forceinline__ void chol_wave_step(double (&v)[MB][MB], double* col, double* pivs, int r, int g, int q,
                                               bool& bad, int JJ, double& pivot) {
    const int j = 8 * PH + JJ;
    constexpr int PN = LAST ? PH + 1 : PH;  // column block of column j + 1
    const int JN = (JJ + 1) & 7;            // its owners' q
    // the pivot comes in a register (read from its lane by the step before); every read of
    // the column is issued before the pivot's arithmetic (all indices are within col), so
    // that their LDS round trips overlap the reciprocal square root
    const double piv = pivot;
    double ci[MB], ck[MB];
#pragma unroll
    for (int m = PH; m < MB; ++m) {
        ci[m] = col[g + 8 * m];
        ck[m] = col[q + 8 * m];
    }
    bad |= !(piv > 0.0);
    if (g == 0 && q == 0) pivs[j] = piv;  // logs are taken after the sweep, off the critical path
    // 1/sqrt(piv): hardware estimate and two Newton steps (relative error ~1 ulp)
    double isq = __builtin_amdgcn_rsq(piv);
    isq = isq * (1.5 - 0.5 * piv * isq * isq);
    isq = isq * (1.5 - 0.5 * piv * isq * isq);
    const double rs = piv * isq;
    const double inv = isq * isq;
    // trailing update a_ik -= a_ij a_kj / a_jj: one side scaled by 1 / a_jj
    double li[MB], lk[MB];
#pragma unroll
    for (int m = PH; m < MB; ++m) {
        const int i = g + 8 * m;
        li[m] = (i > j) ? ci[m] : 0.0;
        const int kk = q + 8 * m;
        lk[m] = (kk > j) ? ck[m] * inv : 0.0;
    }
    if constexpr (PN < MB) {
#pragma unroll
        for (int m = PN; m < MB; ++m) v[m][PN] -= li[m] * lk[PN];
        // the next pivot a_{j+1,j+1}: element (PN, PN) of lane (g, q) = (JN, JN)
        if (j + 1 < r) pivot = lane_value(v[PN][PN], 9 * JN);
        // col is read above before it is written here (one wave: LDS operations in order)
        if (j + 1 < r && q == JN) {
#pragma unroll
            for (int m = PN; m < MB; ++m) col[g + 8 * m] = v[m][PN];
        }
    }
#pragma unroll
    for (int m = PH; m < MB; ++m)
#pragma unroll
        for (int cc = PH; cc <= m; ++cc)
            if (cc != PN) v[m][cc] -= li[m] * lk[cc];
    if (q == JJ) {
#pragma unroll
        for (int m = PH; m < MB; ++m) {
            const int i = g + 8 * m;
            if (i == j) v[m][PH] = rs;
            else if (i > j) v[m][PH] *= isq;
        }
    }
    chol_sync<WS>();
}

// A phase hook that does nothing (hook.template done<PH>(v) runs after every phase that
// completes all its eight columns, with those columns final in v).
struct CholNoHook {
    template <int PH, typename V>
    __device__ __forceinline__ void done(V&) {}
};

template <int MB, int PH, bool WS = false>
struct CholWavePhases {
    // pivot: a_jj of the first column of the phase, in every lane
    template <typename Hook = CholNoHook>
    __device__ __forceinline__ static void run(double (&v)[MB][MB], double* col, double* pivs, int r, int g, int q,
                                               bool& bad, double& pivot, Hook&& hook = Hook{}) {
#pragma unroll 1
        for (int JJ = 0; JJ < 7; ++JJ) {
            if (8 * PH + JJ >= r) return;
            chol_wave_step<MB, PH, false, WS>(v, col, pivs, r, g, q, bad, JJ, pivot);
        }
        if (8 * PH + 7 >= r) return;
        chol_wave_step<MB, PH, true, WS>(v, col, pivs, r, g, q, bad, 7, pivot);
        hook.template done<PH>(v);
        if constexpr (PH + 1 < MB) CholWavePhases<MB, PH + 1, WS>::run(v, col, pivs, r, g, q, bad, pivot, hook);
    }
};


}  // namespace dino
