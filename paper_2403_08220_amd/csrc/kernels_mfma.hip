// BF16 MFMA kernels of the mixed-precision path (gfx950):
//  * fused reverse-mode reduced Jacobian (the display after eq. rb_dino): all layers of
//    the sweep Lambda <- Lambda [+] (Lambda D_l) W_l in one launch, Lambda kept in
//    registers in FP32, products on v_mfma_f32_32x32x16_bf16;
//  * Gauss-Newton Hessian I + B^T B (eq. surrogate_rppgnh) and reduced ppg B^T e
//    (eq. surrogate_rppg, sign as in eq. ppg) per chain, written in FP64 for the
//    Cholesky factorisation;
//  * FP32 forward helpers (input conversion, whitened residual and misfit).
//
// Layout of the sweep. A wave owns 32 columns R = (chain, output) of Lambda^T (width
// rows x 32). One 32x32x16 MFMA takes A (32 x 16) with lane (m, h) holding
// A[m][8h + j], B (16 x 32) with lane (n, h) holding B[8h + j][n], and returns D
// (32 x 32) with lane (n, h), register j holding D[8(j/4) + 4h + j%4][n]. The 8
// registers 8q..8q+7 of a D block therefore hold, for lane (n, h), rows
// 16q + pi(h, jj) with pi(h, jj) = 8(jj/4) + 4h + jj%4 - exactly one B operand of a
// 16-deep K chunk up to the permutation pi of K inside the chunk. The weight tiles
// (the A operands, W_l^T) are packed on the host with the same permutation, so the
// result of one layer feeds the next layer's products without leaving registers.
#include "dino_internal.hpp"
#include "chol_wave.hpp"

namespace dino {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(16))) _Float16 f16x16;

constexpr int JAC_WAVES = 4;          // waves per block of the sweep kernel
constexpr int JAC_TPB = 64 * JAC_WAVES;

__device__ __forceinline__ int pi_row(int h, int jj) { return 8 * (jj >> 2) + 4 * h + (jj & 3); }

// ---------------------------------------------------------------------------------
// Sweep arguments: reverse layers in processing order (output side first). The
// packed tiles of one (layer, output block) work item are contiguous: NT(NMB) tiles
// of 1 KB, of which the first 2*NMB hold the K chunks (zero beyond the layer's K).

struct SweepLayer {
    const float* d;       // gelu'(z) of the layer (C x ldd, zero padded) or null
    int nmb_out;          // output row blocks of 32 (ceil(fan_in / 32))
    int resid;            // Lambda <- Lambda + ...
};

struct SweepArgs {
    int n_cols;           // C * dy
    int dy;
    int w_out;            // fan_in of the output layer (rows of Lambda_L)
    int ldd;              // row length of the d buffers
    int r;                // rows of the final B^T
    int ldb;              // row stride of B (r rounded up to 32)
    int n_layers;
    int n_items;
    const float* Wout;    // output layer weights (d_out x w_out), FP32
    const double* winv;   // Gamma^-1/2 diagonal, one row of dy per request
    const int32_t* rows;  // request row of every chain (null: row 0)
    __hip_bfloat16* B;    // out: C*dy x r, BF16
    SweepLayer layer[15];
    const bf16x8* tiles;  // all work items' tiles, contiguous in processing order
    const float* ones;    // 32 * NMB ones: the d row of layers without an activation
    const float* wout_pk; // output layer rows in the sweep's register order (width-416 kernel)
    int d_out;            // rows of the output layer
};

constexpr int sweep_nt(int nmb) { return (2 * nmb + 3) / 4 * 4; }  // tiles per item, multiple of 4
// LDS ring depth (a power of two): items are copied NBUF - 1 ahead; the ring fits in 150 KB.
constexpr int sweep_nbuf(int nmb) { return sweep_nt(nmb) * 4 <= 150 ? 4 : 2; }

// One 1 KB tile copy global -> LDS (global_load_lds_dwordx4): every lane moves 16 B of
// its own address to lds_base + 16 * lane. Issued from asm so that the compiler's
// LDS-read scheduling is not serialised behind the copy; completion is tracked by
// the explicit vmcnt waits of the kernel (the copy has no VGPR result). The copy reads
// M0 one wait state after the SALU write. M0 is a reserved register that the compiler
// does not treat as clobbered by asm, so its value is saved and restored around the copy.
__device__ __forceinline__ void dma_tile(const void* gsrc, uint32_t lds_base) {
    uint32_t m0_saved;
    asm volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off\n\t"
                 "s_mov_b32 m0, %0"
                 : "=&s"(m0_saved)
                 : "v"(gsrc), "s"(lds_base)
                 : "memory");
}

// Four LDS-DMA copies of 1 KB (lane u*64 + l moves 16 B from base + doff[u]) into the LDS
// region at dm: the gelu' rows of a wave's chains (completion tracked by the kernel's vmcnt
// waits). M0 is saved and restored as in dma_tile.
__device__ __forceinline__ void dma_rows(const float* base, const uint32_t (&doff)[4], uint32_t dm) {
    const uint64_t b = (uint64_t)(uintptr_t)base;
    const uint64_t bu = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32)) << 32) |
                        (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)b);
    uint32_t m0_saved;
    asm volatile("s_mov_b32 %0, m0\n\t"
                 "s_mov_b32 m0, %5\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, %6\n\t"
                 "s_add_u32 m0, %5, 1024\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %2, %6\n\t"
                 "s_add_u32 m0, %5, 2048\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %3, %6\n\t"
                 "s_add_u32 m0, %5, 3072\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %4, %6\n\t"
                 "s_mov_b32 m0, %0"
                 : "=&s"(m0_saved)
                 : "v"(doff[0]), "v"(doff[1]), "v"(doff[2]), "v"(doff[3]), "s"(dm), "s"(bu)
                 : "scc", "memory");
}

#include "sweep_asm.inc"

template <int NMB>
__global__ __launch_bounds__(JAC_TPB) __attribute__((amdgpu_waves_per_eu(1, 1)))
void jac_sweep_bf16_kernel(SweepArgs args) {
    constexpr int NKC = 2 * NMB;          // K chunks per item (MFMAs per item)
    constexpr int NT = sweep_nt(NMB);     // tiles per item (copies per wave: NT / 4)
    constexpr int NBUF = sweep_nbuf(NMB); // ring depth
    constexpr int YOUNGER = (NBUF - 2) * (NT / 4);  // copies of younger items allowed in flight
    extern __shared__ bf16x8 tiles_lds[]; // NBUF buffers x NT tiles x 64 lanes
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nl = lane & 31, h = lane >> 5;
    const int col = (blockIdx.x * JAC_WAVES + wave) * 32 + nl;
    const bool valid = col < args.n_cols;
    const int c = valid ? col / args.dy : 0;
    const int i = valid ? col % args.dy : 0;

    // The residual stream Lambda^T is kept in FP32 without the Gamma^-1/2 row factor
    // (applied when B is written); each 32-row block is the accumulator of its own
    // MFMA chain, updated in place (D layout). Products run on BF16 operands.
    f32x16 lam[NMB];
    {
        const float* wrow = args.Wout + (long)i * args.w_out;
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int row = 32 * mb + 8 * (j >> 2) + 4 * h + (j & 3);
                lam[mb][j] = (valid && row < args.w_out) ? wrow[row] : 0.f;
            }
    }
    const float wi = valid ? (float)args.winv[(long)(args.rows ? args.rows[c] : 0) * args.dy + i] : 0.f;

    // Work items (layer, output block) are walked in lockstep by all waves. Direct
    // global -> LDS copies (global_load_lds_dwordx4) move whole 1 KB tiles (64 lanes x
    // 16 B at a wave-uniform LDS base); every wave copies NT/4 tiles of an item,
    // NBUF - 1 items ahead, into a ring of NBUF buffers.
    const uint32_t lds_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) bf16x8*)tiles_lds;
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);
    auto stage = [&](int item) {
        const bf16x8* src = args.tiles + (long)item * NT * 64;
        const uint32_t dst = lds_base + (uint32_t)((item & (NBUF - 1)) * NT * 64 * 16);
#pragma unroll
        for (int q = 0; q < NT / 4; ++q) {
            const int kc = wave_u + 4 * q;
            dma_tile(src + kc * 64 + lane, __builtin_amdgcn_readfirstlane(dst + (uint32_t)kc * 1024u));
        }
    };
    // Item k is resident once this wave has at most the copies of the NBUF - 2 items
    // younger than k in flight (copies land in issue order) and every wave has passed
    // the barrier. Near the end of the sequence, where fewer younger items exist, the
    // wait drains everything.
    auto wait_for = [&](int k) {
        if (k + NBUF - 2 <= args.n_items - 1) asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(YOUNGER) : "memory");
        else asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
    };

    for (int k = 0; k < NBUF - 1 && k < args.n_items; ++k) stage(k);
    wait_for(0);
    __hip_bfloat16* brow = args.B + (long)col * args.ldb;

    int item = 0;
    for (int li = 0; li < args.n_layers; ++li) {
        const SweepLayer L = args.layer[li];
        const bool last = (li == args.n_layers - 1);
        // B operands: bf16(d * Lambda) for every K chunk of this layer
        bf16x8 bop[NKC];
        if (L.d) {
            const float4* drow = reinterpret_cast<const float4*>(L.d + (long)c * args.ldd + 4 * h);
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const float4 d0 = drow[8 * mb + 4 * q];
                    const float4 d1 = drow[8 * mb + 4 * q + 2];
                    const float dv[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) bop[2 * mb + q][jj] = (__bf16)(lam[mb][8 * q + jj] * dv[jj]);
                    __builtin_amdgcn_sched_barrier(0);  // keep only one block's gelu' values live
                }
        } else {
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) bop[2 * mb + q][jj] = (__bf16)lam[mb][8 * q + jj];
        }
#pragma unroll
        for (int mob = 0; mob < NMB; ++mob) {
            if (mob < L.nmb_out) {
                if (item + NBUF - 1 < args.n_items) stage(item + NBUF - 1);
                const bf16x8* cur = tiles_lds + (long)(item & (NBUF - 1)) * NT * 64 + lane;
                if (!L.resid)
#pragma unroll
                    for (int j = 0; j < 16; ++j) lam[mob][j] = 0.f;
#pragma unroll
                for (int kc = 0; kc < NKC; ++kc)
                    lam[mob] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cur[kc * 64], bop[kc], lam[mob], 0, 0, 0);
                const f32x16& acc = lam[mob];
                if (last && valid) {
                    // B[col][m] = winv_i Lambda_0^T[m][col]; rows padded to ldb (a multiple of
                    // 32), so whole blocks are written with 8-byte streaming stores
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int m0 = 32 * mob + 8 * b + 4 * h;
                        uint64_t v = 0;
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            v |= (uint64_t)__builtin_bit_cast(uint16_t, __float2bfloat16(wi * acc[4 * b + t])) << (16 * t);
                        __builtin_nontemporal_store(v, reinterpret_cast<uint64_t*>(brow + m0));
                    }
                }
                ++item;
                if (item < args.n_items) wait_for(item);
            }
        }
        // rows beyond this layer's output are zero (no stale values when widths shrink)
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb)
            if (mb >= L.nmb_out)
#pragma unroll
                for (int j = 0; j < 16; ++j) lam[mb][j] = 0.f;
    }
}

// The width-416 instance (13 row blocks, 26 K chunks): every layer is one asm block
// (sweep_layer13) that runs its items with the tile ring protocol of the kernel above
// (copies three items ahead, vmcnt + barrier before an item is read), so that the
// reads of an item overlap the last MFMAs of the previous one and no compiler-placed
// code runs between items. Lambda stays in VGPRs; the B operands live in AGPRs. Layers
// without an activation multiply by a row of ones, so that every layer takes the same
// path.
__global__ __launch_bounds__(JAC_TPB) __attribute__((amdgpu_waves_per_eu(1, 1)))
void jac_sweep13_kernel(SweepArgs args) {
    constexpr int NMB = 13, NKC = 26, NT = 28, NBUF = 4;
    static_assert(sweep_nt(NMB) == NT && sweep_nbuf(NMB) == NBUF, "ring layout of the width-416 sweep");
    constexpr uint32_t ITEM = NT * 1024;  // bytes per item
    extern __shared__ bf16x8 tiles_lds[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nl = lane & 31, h = lane >> 5;
    const int col = (blockIdx.x * JAC_WAVES + wave) * 32 + nl;
    const bool valid = col < args.n_cols;
    const int c = valid ? col / args.dy : 0;
    const int i = valid ? col % args.dy : 0;

    // Lambda_L^T = the output layer's rows, from the packed copy: one 16-byte load per
    // (row block, register quad), 1 KB contiguous per wave. Columns past n_cols compute
    // with output 0 and are never written.
    f32x16 lam[NMB];
    {
        const float4* wp = reinterpret_cast<const float4*>(args.wout_pk) + (long)i * 2 + h;
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
            for (int jq = 0; jq < 4; ++jq) {
                const float4 v = wp[(long)(mb * 4 + jq) * args.d_out * 2];
                lam[mb][4 * jq] = v.x;
                lam[mb][4 * jq + 1] = v.y;
                lam[mb][4 * jq + 2] = v.z;
                lam[mb][4 * jq + 3] = v.w;
            }
    }
    const float wi = valid ? (float)args.winv[(long)(args.rows ? args.rows[c] : 0) * args.dy + i] : 0.f;

    const uint32_t lds_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) bf16x8*)tiles_lds;
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);

    // gelu' rows: when the wave's 32 columns span at most two chains, the wave's two rows
    // (416 FP32 each) of a layer are copied into the wave's 4 KB LDS region, chunk k of
    // 16 B (row k / 104) from lane k % 64 of copy k / 64: the first layer's here, every
    // later layer's by the layer block before it; otherwise every layer reads its rows
    // from global memory
    const int col0 = (blockIdx.x * JAC_WAVES + wave_u) * 32;
    const int c_first = col0 / args.dy;
    const int c_last = min(col0 + 31, args.n_cols - 1) / args.dy;
    const bool staged = col0 < args.n_cols && c_last - c_first <= 1;
    uint32_t doff[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int kk = min(u * 64 + lane, 207);
        const int row = kk / 104;
        doff[u] = (uint32_t)(min(c_first + row, c_last) * args.ldd * 4 + (kk - row * 104) * 16);
    }
    const uint32_t dm = __builtin_amdgcn_readfirstlane(lds_base + NBUF * ITEM + (uint32_t)wave_u * 4096u);
    // the lane's row in the region as an LDS byte address, plus the lane's 16-byte offset
    const uint32_t vd = dm + (uint32_t)((valid ? c - c_first : 0) * 1664 + 16 * h);
    // (copied before the tiles: the prologue's wait for item 0 also completes them)
    if (staged && args.n_layers > 0 && args.layer[0].d) dma_rows(args.layer[0].d, doff, dm);

    for (int k = 0; k < NBUF - 1 && k < args.n_items; ++k) {
        const bf16x8* src = args.tiles + (long)k * NT * 64;
#pragma unroll
        for (int q = 0; q < NT / 4; ++q) {
            const int kc = wave_u + 4 * q;
            dma_tile(src + kc * 64 + lane, __builtin_amdgcn_readfirstlane(lds_base + (uint32_t)k * ITEM + kc * 1024u));
        }
    }
    if (NBUF - 2 <= args.n_items - 1) asm volatile("s_waitcnt vmcnt(14)\n\ts_barrier" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");

    const uint32_t sb = __builtin_amdgcn_readfirstlane(lds_base);
    const uint64_t tb = (uint64_t)(uintptr_t)args.tiles;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)tb);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(tb >> 32));
    const uint32_t sw = __builtin_amdgcn_readfirstlane((uint32_t)wave_u * 1024u);
    bf16x8 zero;
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) zero[jj] = (__bf16)0.f;

    int item = 0;
    bool formed = false;  // the previous layer block formed this layer's operands
    bf16x8 bop[NKC];
    for (int li = 0; li < args.n_layers; ++li) {
        const SweepLayer L = args.layer[li];
        // B operands bf16(d * Lambda) of this layer, unless the block before formed them
        if (!formed) {
            if (staged && L.d) sweep_form13_lds(lam, bop, vd);
            else sweep_form13_global(lam, bop, (L.d ? L.d + (long)c * args.ldd : args.ones) + 4 * h);
        }
        const uint32_t sc = __builtin_amdgcn_readfirstlane(lds_base + (uint32_t)(item & (NBUF - 1)) * ITEM);
        // every scalar operand of the block is wave-uniform; readfirstlane places it in an SGPR
        const uint32_t n_u =
            __builtin_amdgcn_readfirstlane(((uint32_t)L.nmb_out & 0xffu) | ((uint32_t)(L.resid == 0) << 8));
        const int32_t tl_u = __builtin_amdgcn_readfirstlane(args.n_items - (NBUF - 1) - item);
        const uint32_t so_u = __builtin_amdgcn_readfirstlane((uint32_t)(item + NBUF - 1) * ITEM);
        const uint32_t se_u = __builtin_amdgcn_readfirstlane(sb + NBUF * ITEM);
        const uint32_t sz_u = __builtin_amdgcn_readfirstlane(sb + (NBUF - 1) * ITEM);
        const float* dnext = li + 1 < args.n_layers ? args.layer[li + 1].d : nullptr;
        const uint32_t df_u = __builtin_amdgcn_readfirstlane((staged && dnext) ? 1u : 0u);
        // the block forms the next layer's operands itself when its gelu' rows are staged and
        // every output block runs
        const bool fuse = staged && dnext && L.nmb_out == NMB;
        const uint32_t ff_u = __builtin_amdgcn_readfirstlane(fuse ? 1u : 0u);
        const uint64_t dsb = (uint64_t)(uintptr_t)(dnext ? dnext : args.ones);
        // (readfirstlane returns int: each half goes through uint32_t so that the low half is
        // not sign-extended into the high one)
        const uint64_t dsb_u = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(dsb >> 32)) << 32) |
                               (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)dsb);
        sweep_layer13(lam, bop, n_u, tl_u, sc, so_u, lo, hi, sb, se_u, sz_u, sw, (uint32_t)lane * 16u, zero,
                      df_u, dsb_u, dm, doff, ff_u, vd);
        formed = fuse;
        item += L.nmb_out;
    }
    // B[col][m] = winv_i Lambda_0^T[m][col] (rows of ldb = 32 * nmb_last BF16). The wave's 32
    // rows are one contiguous block of B: they are assembled in LDS (the ring is no longer
    // read once every wave has passed the barrier below) and written with 16-byte stores.
    __syncthreads();
    {
        const int ldb = args.ldb;
        const int nmb_last = args.layer[args.n_layers - 1].nmb_out;
        char* stage_lds = reinterpret_cast<char*>(tiles_lds) + (size_t)wave * 64 * ldb;
#pragma unroll
        for (int mob = 0; mob < NMB; ++mob) {
            if (mob < nmb_last) {
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int m0 = 32 * mob + 8 * b + 4 * h;
                    uint64_t v = 0;
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        v |= (uint64_t)__builtin_bit_cast(uint16_t, __float2bfloat16(wi * lam[mob][4 * b + t])) << (16 * t);
                    *reinterpret_cast<uint64_t*>(stage_lds + ((size_t)nl * ldb + m0) * 2) = v;
                }
            }
        }
        __syncthreads();
        const int col0 = (blockIdx.x * JAC_WAVES + wave) * 32;
        const int rows = min(32, args.n_cols - col0);
        const int chunks = rows * ldb / 8;  // 16-byte chunks of the wave's block
        char* dst = reinterpret_cast<char*>(args.B + (long)col0 * ldb);
        typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;
        for (int e = lane; e < chunks; e += 64)
            __builtin_nontemporal_store(*reinterpret_cast<const u32x4*>(stage_lds + (size_t)e * 16),
                                        reinterpret_cast<u32x4*>(dst + (size_t)e * 16));
    }
}

// ---------------------------------------------------------------------------------
// Per chain: A = I + B^T B (lower triangle, FP64, into the factor slot) and
// g = B^T e, with B the chain's dy x r whitened Jacobian (BF16) and e the whitened
// residual (FP32). B^T is staged in LDS (r_pad x dy_pad) so that every MFMA operand
// is one 16-byte read.
constexpr int HES_TPB = 256;

// Whitened residual e_i = Gamma^-1/2 (f_i - y_i) of chain c into es (FP32; zero where the
// noise variance is infinite) and the misfit phi_c = |e|^2 / 2 summed in FP64 (Sec. 5.1).
// f: the FP32 network output; y, winv: per request row. Called by all HES_TPB threads;
// red holds HES_TPB / 64 doubles; es is complete after the call.
__device__ __forceinline__ void residual_into(int c, int dy, const float* __restrict__ f,
                                              const double* __restrict__ y_rows,
                                              const double* __restrict__ winv_rows, const int32_t* __restrict__ rows,
                                              float* es, double* red, double* __restrict__ phi) {
    const int tid = threadIdx.x;
    const long row = rows ? rows[c] : 0;
    const double* y = y_rows + row * dy;
    const double* winv = winv_rows + row * dy;
    double part = 0.0;
    for (int i = tid; i < dy; i += HES_TPB) {
        const double w = winv[i];
        const double v = (w == 0.0) ? 0.0 : ((double)f[(long)c * dy + i] - y[i]) * w;
        es[i] = (float)v;
        part += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if ((tid & 63) == 0) red[tid >> 6] = part;
    __syncthreads();
    if (tid == 0 && phi) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < HES_TPB / 64; ++k) t += red[k];
        phi[c] = 0.5 * t;
    }
}

__global__ __launch_bounds__(HES_TPB) void hess_bf16_kernel(int dy, int r, int ldb, int dy_pad, int ldt,
                                                            const __hip_bfloat16* __restrict__ B,
                                                            const float* __restrict__ f, const double* y_rows,
                                                            const double* winv_rows, const int32_t* rows,
                                                            double* __restrict__ phi, double* A, long strideA,
                                                            const int32_t* slot, int slot_xor, long slot_stride,
                                                            double* __restrict__ g) {
    extern __shared__ __hip_bfloat16 bt[];  // r_pad x ldt, then e (dy floats)
    __shared__ double red[HES_TPB / 64];
    const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nmb = (r + 31) / 32;
    const int r_pad = nmb * 32;
    const __hip_bfloat16* Bc = B + (long)c * dy * ldb;
    float* es = reinterpret_cast<float*>(bt + (long)r_pad * ldt);
    // transpose into LDS: bt[j][i] = B[i][j], zero padded
    for (int e2 = tid; e2 < r_pad * dy_pad; e2 += HES_TPB) {
        const int j = e2 / dy_pad, ii = e2 % dy_pad;
        bt[(long)j * ldt + ii] = (j < r && ii < dy) ? Bc[(long)ii * ldb + j] : __float2bfloat16(0.f);
    }
    residual_into(c, dy, f, y_rows, winv_rows, rows, es, red, phi);  // ends with a barrier
    // gradient g_j = sum_i B[i][j] e[i]
    for (int j = tid; j < r; j += HES_TPB) {
        double acc = 0.0;
        for (int ii = 0; ii < dy; ++ii) acc += (double)__bfloat162float(bt[(long)j * ldt + ii]) * (double)es[ii];
        g[(long)c * r + j] = acc;
    }
    if (!A) return;  // misfit and ppg only (the MALA baseline forms no metric)
    double* Ac = A + (long)c * strideA + (slot ? (long)(slot[c] ^ slot_xor) * slot_stride : 0);
    const int nl = lane & 31, h = lane >> 5;
    const int nkc = dy_pad / 16;
    // lower 32x32 blocks (bj >= bk) distributed over the waves
    const int nblocks = nmb * (nmb + 1) / 2;
    for (int bidx = wave; bidx < nblocks; bidx += HES_TPB / 64) {
        int bj = 0;
        while ((bj + 1) * (bj + 2) / 2 <= bidx) ++bj;
        const int bk = bidx - bj * (bj + 1) / 2;
        f32x16 acc;
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = 0.f;
        for (int kc = 0; kc < nkc; ++kc) {
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(bt + (long)(32 * bj + nl) * ldt + 16 * kc + 8 * h);
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(bt + (long)(32 * bk + nl) * ldt + 16 * kc + 8 * h);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        const int col = 32 * bk + nl;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int row = 32 * bj + 8 * (j >> 2) + 4 * h + (j & 3);
            if (row < r && col < r && col <= row) Ac[(long)row * r + col] = (double)acc[j] + (row == col ? 1.0 : 0.0);
        }
    }
}

// The same Hessian, ppg and misfit for shapes whose B^T does not fit one block's LDS
// (reduced dimensions and observation counts of several hundred): one block per chain and
// lower 64 x 64 tile (bi >= bk) of I + B^T B, B streamed through LDS in chunks of 64 rows
// (observed outputs), transposed as they are staged. Each wave forms one 32 x 32 sub-tile.
// Diagonal tiles also form the ppg of their 64 columns; tile (0, 0) writes the misfit. The
// products, and their order over the outputs, are those of hess_bf16_kernel, so the two
// agree bit for bit where both apply. Work items are laid out so that the tiles of one
// chain run on one XCD and share its L2 copy of B.
constexpr int HT_CH = 64;
__global__ __launch_bounds__(HES_TPB) void hess_bf16_tiled_kernel(int n, int dy, int r, int ldb, int ntile,
                                                                  const __hip_bfloat16* __restrict__ B,
                                                                  const float* __restrict__ f, const double* y_rows,
                                                                  const double* winv_rows, const int32_t* rows,
                                                                  double* __restrict__ phi, double* A, long strideA,
                                                                  const int32_t* slot, int slot_xor, long slot_stride,
                                                                  double* __restrict__ g) {
    __shared__ __align__(16) __hip_bfloat16 ti[64 * (HT_CH + 8)];
    __shared__ __align__(16) __hip_bfloat16 tk[64 * (HT_CH + 8)];
    __shared__ float es[1024];
    __shared__ double red[HES_TPB / 64];
    const long total = (long)n * ntile;
    const long per = (total + 7) / 8;
    const long w = (long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (w >= total) return;
    const int c = (int)(w / ntile), t = (int)(w - (long)(w / ntile) * ntile);
    int bi = 0;
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    const int bk = t - bi * (bi + 1) / 2;
    const bool diag = bi == bk;
    if (!A && !diag) return;  // ppg and misfit only (the MALA baseline forms no metric)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nl = lane & 31, h = lane >> 5, wi = wave & 1, wk = wave >> 1;
    const __hip_bfloat16* Bc = B + (long)c * dy * ldb;
    const __hip_bfloat16* tkp = diag ? ti : tk;
    if (diag) residual_into(c, dy, f, y_rows, winv_rows, rows, es, red, (bi == 0) ? phi : nullptr);
    const bool mine = A && !(diag && wk > wi);  // the diagonal tile's upper sub-tile is not formed
    f32x16 acc;
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = 0.f;
    double gacc = 0.0;
    for (int k0 = 0; k0 < dy; k0 += HT_CH) {
        __syncthreads();  // the previous chunk is consumed
        for (int e = tid; e < HT_CH * 8; e += HES_TPB) {
            const int kk = e >> 3, c8 = (e & 7) * 8, k = k0 + kk;
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                if (side == 1 && diag) break;
                const int col = 64 * (side ? bk : bi) + c8;
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (k < dy && col < ldb) v = *reinterpret_cast<const uint4*>(Bc + (long)k * ldb + col);
                const __hip_bfloat16* pv = reinterpret_cast<const __hip_bfloat16*>(&v);
                __hip_bfloat16* dst = side ? tk : ti;
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    dst[(c8 + j) * (HT_CH + 8) + kk] = (col + j < r) ? pv[j] : __float2bfloat16(0.f);
            }
        }
        __syncthreads();
        if (diag && tid < 64) {
            const int kn = min(HT_CH, dy - k0);
            for (int kk = 0; kk < kn; ++kk)
                gacc += (double)__bfloat162float(ti[tid * (HT_CH + 8) + kk]) * (double)es[k0 + kk];
        }
        if (mine) {
#pragma unroll
            for (int s = 0; s < HT_CH / 16; ++s) {
                if (k0 + 16 * s >= dy) break;
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(ti + (32 * wi + nl) * (HT_CH + 8) + 16 * s + 8 * h);
                const bf16x8 b = *reinterpret_cast<const bf16x8*>(tkp + (32 * wk + nl) * (HT_CH + 8) + 16 * s + 8 * h);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
            }
        }
    }
    if (diag && tid < 64 && 64 * bi + tid < r) g[(long)c * r + 64 * bi + tid] = gacc;
    if (!mine) return;
    double* Ac = A + (long)c * strideA + (slot ? (long)(slot[c] ^ slot_xor) * slot_stride : 0);
    const int col = 64 * bk + 32 * wk + nl;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int row = 64 * bi + 32 * wi + 8 * (j >> 2) + 4 * h + (j & 3);
        if (row < r && col < r && col <= row) Ac[(long)row * r + col] = (double)acc[j] + (row == col ? 1.0 : 0.0);
    }
}

// x (double) -> xf (float)
__global__ void to_float_kernel(long n, const double* __restrict__ x, float* __restrict__ xf) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        xf[e] = (float)x[e];
}

__global__ void to_double_kernel(long n, const float* __restrict__ xf, double* __restrict__ x) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        x[e] = (double)xf[e];
}

// ---------------------------------------------------------------------------------
// Host side.

// The sweep kernel instance (its NMB) used for a network whose widest reverse
// operand spans nmb row blocks of 32.
int sweep_template_nmb(int nmb) {
    if (nmb <= 2) return 2;
    if (nmb <= 4) return 4;
    if (nmb <= 7) return 7;
    if (nmb <= 13) return 13;
    return 16;
}

// Row blocks of 32 that the sweep must hold: the widest of r and the hidden layers.
static int sweep_blocks(const dino_ctx* ctx) {
    int m = (ctx->r_in + 31) / 32;
    for (size_t l = 0; l + 1 < ctx->layers.size(); ++l) {
        m = std::max(m, (ctx->layers[l].fan_in + 31) / 32);
        m = std::max(m, (ctx->layers[l].fan_out + 31) / 32);
    }
    return m;
}

int sweep_nmb(const dino_ctx* ctx) { return sweep_template_nmb(sweep_blocks(ctx)); }

bool sweep_width_ok(const dino_ctx* ctx) { return sweep_blocks(ctx) <= 16; }

// Pack A = W^T tiles for one layer W (fan_out x fan_in) for the sweep instance nmb_t:
// work item mo (output rows 32 mo .. 32 mo + 31) holds sweep_nt(nmb_t) tiles; tile kc,
// lane (m, h), slot jj = W[16 kc + pi(h, jj)][32 mo + m] (zero outside W).
void pack_sweep_tiles(const std::vector<double>& W, int fan_out, int fan_in, int nmb_t,
                      std::vector<uint16_t>& out, int& nmb_out) {
    nmb_out = (fan_in + 31) / 32;
    const int nt = sweep_nt(nmb_t);
    out.assign((size_t)nmb_out * nt * 64 * 8, 0);
    for (int mo = 0; mo < nmb_out; ++mo)
        for (int kc = 0; kc < 2 * nmb_t; ++kc)
            for (int lane = 0; lane < 64; ++lane) {
                const int m = lane & 31, h = lane >> 5;
                for (int jj = 0; jj < 8; ++jj) {
                    const int k = 16 * kc + 8 * (jj >> 2) + 4 * h + (jj & 3);
                    const int n = 32 * mo + m;
                    float v = 0.f;
                    if (k < fan_out && n < fan_in) v = (float)W[(size_t)k * fan_in + n];
                    uint32_t u;  // round to nearest even BF16
                    std::memcpy(&u, &v, 4);
                    u += 0x7FFFu + ((u >> 16) & 1u);
                    out[(((size_t)mo * nt + kc) * 64 + lane) * 8 + jj] = (uint16_t)(u >> 16);
                }
            }
}

void pack_sweep_wout(const std::vector<double>& W, int fan_out, int fan_in, int nmb_t, std::vector<float>& out) {
    out.assign((size_t)nmb_t * 4 * fan_out * 8, 0.f);
    for (int mb = 0; mb < nmb_t; ++mb)
        for (int jq = 0; jq < 4; ++jq)
            for (int i = 0; i < fan_out; ++i)
                for (int hh = 0; hh < 2; ++hh)
                    for (int t = 0; t < 4; ++t) {
                        const int row = 32 * mb + 8 * jq + 4 * hh + t;
                        if (row < fan_in)
                            out[(((size_t)mb * 4 + jq) * fan_out + i) * 8 + 4 * hh + t] = (float)W[(size_t)i * fan_in + row];
                    }
}

template <int NMB>
static void launch_sweep_t(const SweepArgs& a, hipStream_t st) {
    const size_t lds = (size_t)sweep_nbuf(NMB) * sweep_nt(NMB) * 64 * sizeof(bf16x8);
    static bool attr = false;
    if (!attr) {
        DINO_HIP(hipFuncSetAttribute((const void*)jac_sweep_bf16_kernel<NMB>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr = true;
    }
    const int blocks = (a.n_cols + 32 * JAC_WAVES - 1) / (32 * JAC_WAVES);
    hipLaunchKernelGGL(jac_sweep_bf16_kernel<NMB>, dim3(blocks), dim3(JAC_TPB), lds, st, a);
    DINO_HIP(hipGetLastError());
}

static void launch_sweep13(const SweepArgs& a, hipStream_t st) {
    // tile ring + one 4 KB gelu' region per wave
    const size_t lds = (size_t)sweep_nbuf(13) * sweep_nt(13) * 64 * sizeof(bf16x8) + JAC_WAVES * 4096;
    static bool attr = false;
    if (!attr) {
        DINO_HIP(hipFuncSetAttribute((const void*)jac_sweep13_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds));
        attr = true;
    }
    const int blocks = (a.n_cols + 32 * JAC_WAVES - 1) / (32 * JAC_WAVES);
    hipLaunchKernelGGL(jac_sweep13_kernel, dim3(blocks), dim3(JAC_TPB), lds, st, a);
    DINO_HIP(hipGetLastError());
}

void launch_sweep_bf16(dino_problem* p, int n, const float* d32, int ldd, __hip_bfloat16* Bout, hipStream_t st) {
    const dino_ctx* ctx = p->ctx;
    const int L = (int)ctx->layers.size();
    const int nmb_t = sweep_nmb(ctx);
    SweepArgs a{};
    a.n_cols = n * p->d_y;
    a.dy = p->d_y;
    a.w_out = ctx->layers[L - 1].fan_in;
    a.ldd = ldd;
    a.r = p->r;
    a.ldb = (p->r + 31) / 32 * 32;
    a.Wout = ctx->layers[L - 1].W32;
    a.winv = p->winv;
    a.rows = p->meta.row;
    a.B = Bout;
    a.n_layers = L - 1;
    a.tiles = reinterpret_cast<const bf16x8*>(ctx->sweep_tiles);
    a.ones = ctx->sweep_ones;
    a.wout_pk = ctx->sweep_wout;
    a.d_out = ctx->layers[L - 1].fan_out;
    DINO_REQUIRE(ldd >= 32 * nmb_t, DINO_EINVAL, "gelu' buffer rows shorter than the sweep width");
    int act = p->n_act, items = 0;
    const int nt = sweep_nt(nmb_t);
    for (int k = 0; k < L - 1; ++k) {
        const int l = L - 2 - k;
        const Layer& ly = ctx->layers[l];
        SweepLayer& s = a.layer[k];
        s.nmb_out = (ly.fan_in + 31) / 32;
        s.resid = ly.kind == DINO_LAYER_RESID ? 1 : 0;
        if (ly.kind != DINO_LAYER_LINEAR) {
            --act;
            s.d = d32 + (long)act * p->C * ldd;
        } else {
            s.d = nullptr;
        }
        items += s.nmb_out;
    }
    a.n_items = items;
    if (nmb_t == 2) launch_sweep_t<2>(a, st);
    else if (nmb_t == 4) launch_sweep_t<4>(a, st);
    else if (nmb_t == 7) launch_sweep_t<7>(a, st);
    else if (nmb_t == 13) launch_sweep13(a, st);
    else launch_sweep_t<16>(a, st);
}

// Observation-space Gram matrix I + B B^T (d_y x d_y, lower 32x32 blocks by MFMA, FP32
// accumulation, written in FP64 for the Cholesky factorisation) and the reduced ppg
// g = B^T e (FP64), one block per chain. The rows of B are the A and B operands of
// v_mfma_f32_32x32x16_bf16 as they are (K = the reduced index): no transpose.
__global__ __launch_bounds__(HES_TPB) void gram_bf16_kernel(int dy, int r, int ldb, int dy_pad, int k_pad, int ldt,
                                                            const __hip_bfloat16* __restrict__ B,
                                                            const float* __restrict__ f, const double* y_rows,
                                                            const double* winv_rows, const int32_t* rows,
                                                            double* __restrict__ phi, double* A, long strideA,
                                                            const int32_t* slot, int slot_xor, long slot_stride,
                                                            double* __restrict__ g) {
    extern __shared__ __hip_bfloat16 bs[];  // dy_pad x ldt, then e (dy floats)
    __shared__ double red[HES_TPB / 64];
    const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const __hip_bfloat16* Bc = B + (long)c * dy * ldb;
    float* es = reinterpret_cast<float*>(bs + (long)dy_pad * ldt);
    // 16-byte moves of 8 BF16 values; columns at or beyond r are zero, as are rows beyond dy
    const int k8 = k_pad / 8;
    for (int e2 = tid; e2 < dy_pad * k8; e2 += HES_TPB) {
        const int i = e2 / k8, j8 = 8 * (e2 - i * k8);
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (i < dy) {
            if (j8 + 8 <= r) {
                v = *reinterpret_cast<const uint4*>(Bc + (long)i * ldb + j8);
            } else {
                __hip_bfloat16 t[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) t[q] = (j8 + q < r) ? Bc[(long)i * ldb + j8 + q] : __float2bfloat16(0.f);
                v = *reinterpret_cast<const uint4*>(t);
            }
        }
        *reinterpret_cast<uint4*>(bs + (long)i * ldt + j8) = v;
    }
    residual_into(c, dy, f, y_rows, winv_rows, rows, es, red, phi);  // ends with a barrier
    for (int j = tid; j < r; j += HES_TPB) {
        double acc = 0.0;
#pragma unroll 4
        for (int i = 0; i < dy; ++i) acc += (double)__bfloat162float(bs[(long)i * ldt + j]) * (double)es[i];
        g[(long)c * r + j] = acc;
    }
    if (!A) return;  // misfit and ppg only (the MALA baseline forms no metric)
    double* Ac = A + (long)c * strideA + (slot ? (long)(slot[c] ^ slot_xor) * slot_stride : 0);
    const int nl = lane & 31, h = lane >> 5;
    const int nmb = dy_pad / 32, nkc = k_pad / 16;
    const int nblocks = nmb * (nmb + 1) / 2;
    for (int bidx = wave; bidx < nblocks; bidx += HES_TPB / 64) {
        int bi = 0;
        while ((bi + 1) * (bi + 2) / 2 <= bidx) ++bi;
        const int bk = bidx - bi * (bi + 1) / 2;
        f32x16 acc;
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = 0.f;
        for (int kc = 0; kc < nkc; ++kc) {
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(bs + (long)(32 * bi + nl) * ldt + 16 * kc + 8 * h);
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(bs + (long)(32 * bk + nl) * ldt + 16 * kc + 8 * h);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        const int col = 32 * bk + nl;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int row = 32 * bi + 8 * (j >> 2) + 4 * h + (j & 3);
            if (row < dy && col <= row) Ac[(long)row * dy + col] = (double)acc[j] + (row == col ? 1.0 : 0.0);
        }
    }
}

void launch_gram_bf16(dino_problem* p, int n, const __hip_bfloat16* B, const float* f, double* phi, double* A,
                      long strideA, const int32_t* slot, int slot_xor, long slot_stride, double* g, hipStream_t st) {
    const int r = p->r, dy = p->d_y;
    const int dy_pad = (dy + 31) / 32 * 32;
    const int k_pad = (r + 15) / 16 * 16;
    const int ldt = k_pad + 8;  // 16-byte aligned rows, shifted banks
    const size_t lds = (size_t)dy_pad * ldt * sizeof(__hip_bfloat16) + (size_t)dy * sizeof(float);
    DINO_REQUIRE(lds <= 160 * 1024 - 64, DINO_EINVAL, "d_y x r too large for the LDS-staged Gram matrix");
    static bool attr = false;
    if (!attr) {
        DINO_HIP(hipFuncSetAttribute((const void*)gram_bf16_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     160 * 1024 - 64));
        attr = true;
    }
    hipLaunchKernelGGL(gram_bf16_kernel, dim3(n), dim3(HES_TPB), lds, st, dy, r, (r + 31) / 32 * 32, dy_pad, k_pad,
                       ldt, B, f, p->y, p->winv, p->meta.row, phi, A, strideA, slot, slot_xor, slot_stride, g);
    DINO_HIP(hipGetLastError());
}

// Column `lane` of D = L_bb^-1 for one diagonal block of the factor (Lc: the block in
// LDS, column-major with stride 32; entries at or past nb are padded with the identity
// here, so that NS branch-free steps of right-looking substitution serve any nb <= NS),
// written into the strictly upper triangle of the factor's block: D[k][lane] at row
// b0 + lane, column b0 + k (row stride dy). Lane k holds 1 / L_kk. Column k + 1 is loaded
// while column k is applied; after each step an empty asm statement takes the updated
// entries as operands and clobbers memory, so that the compiler neither sinks a step's
// products below later steps nor hoists later columns' loads above it.
template <int NS>
__device__ __forceinline__ void invert_diag_block(double* Lc, int nb, int lane, double* a, int dy, int b0) {
    if (nb < NS) {
        for (int e = lane; e < NS * NS; e += 64) {
            const int k = e / NS, i = e - k * NS;
            if (i >= nb || k >= nb) Lc[k * 32 + i] = (i == k) ? 1.0 : 0.0;
        }
    }
    const double rl = 1.0 / Lc[(lane % NS) * 33];
    double d[NS], col[2][NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) d[k] = (k == lane) ? 1.0 : 0.0;
#pragma unroll
    for (int i = 1; i < NS; ++i) col[0][i] = Lc[i];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
#pragma unroll
        for (int i = k + 2; i < NS; ++i) col[(k + 1) & 1][i] = Lc[(k + 1) * 32 + i];
        d[k] *= lane_value(rl, k);
#pragma unroll
        for (int i = k + 1; i < NS; ++i) d[i] -= col[k & 1][i] * d[k];
#pragma unroll
        for (int i = k; i < NS; ++i) asm volatile("" : "+v"(d[i]));
        asm volatile("" ::: "memory");
    }
    if (lane < nb) {
#pragma unroll
        for (int k = 1; k < NS; ++k)
            if (k > lane && k < nb) a[(long)(b0 + lane) * dy + b0 + k] = d[k];
    }
}

// Phase hook of the fused kernel's factorisation: once the phase that completes diagonal
// block b (columns 32 b .. 32 b + 31) is done, the first wave copies the block to LDS
// (column-major) and raises ready[b]; another wave inverts it while the factorisation
// goes on.
template <int MB>
struct DiagBlockPublish {
    double* Ld;
    int* ready;
    int dy, g, q;
    template <int PH>
    __device__ __forceinline__ void done(double (&v)[MB][MB]) {
        if constexpr ((PH & 3) == 3) {
            constexpr int b = PH / 4;
            if (32 * b + 32 <= dy) {
#pragma unroll
                for (int m = 4 * b; m < 4 * b + 4; ++m)
#pragma unroll
                    for (int cc = 4 * b; cc <= m; ++cc) {
                        const int i = g + 8 * m, kk = q + 8 * cc;
                        if (kk <= i) Ld[b * 1024 + (kk & 31) * 32 + (i & 31)] = v[m][cc];
                    }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // the block is in LDS first
                if (g == 0 && q == 0) __hip_atomic_store(ready + b, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
};

// Observation-space Gram matrix and its Cholesky factor in one launch, one block per
// chain: the block stages the chain's B, forms the residual, the misfit and g = B^T e as
// gram_bf16_kernel does, accumulates the lower 32 x 32 blocks of B B^T by MFMA in
// registers, writes B B^T (FP32, the accumulation precision) over B's LDS, and its first
// wave factorises K = I + B B^T in FP64 registers (the identity added in FP64; the
// single-wave column steps), so that K never leaves LDS and the factor equals that of the
// separate Gram and factor kernels bit for bit. Writes the factor (lower triangle, row stride d_y), log det K / 2
// and the pivot flag. d_y <= 8 MB. With dinv the kernel also inverts the diagonal blocks
// of 32 rows (D_b = L_bb^-1, written into the strictly upper triangle of the factor's
// block (b, b); the solves of the dual proposal and acceptance read it there and form
// its diagonal, 1 / L_jj, themselves): wave b + 1 inverts full block b as soon as the
// factorisation has passed it (d_y <= 104: at most three full blocks), the first wave
// inverts a short last block after the factorisation.
template <int MB>
__global__ __launch_bounds__(HES_TPB) __attribute__((amdgpu_waves_per_eu(2, 2)))
void gram_chol_bf16_kernel(int dy, int r, int ldb, int dy_pad, int k_pad, int ldt,
                           const __hip_bfloat16* __restrict__ B, const float* __restrict__ f, const double* y_rows,
                           const double* winv_rows, const int32_t* rows, double* __restrict__ phi, double* A,
                           long strideA, const int32_t* slot, int slot_xor, long slot_stride, double* __restrict__ g,
                           double* __restrict__ logdet, int32_t* __restrict__ ok, int dinv) {
    extern __shared__ __hip_bfloat16 bs[];  // dy_pad x ldt B, then e (dy floats); K (FP32) over B afterwards
    __shared__ double red[HES_TPB / 64];
    __shared__ double col[8 * MB];
    __shared__ double pivs[8 * MB];
    __shared__ int dready[4];
    const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < 4) dready[tid] = 0;  // ordered before the flags by the barriers below
    const __hip_bfloat16* Bc = B + (long)c * dy * ldb;
    float* es = reinterpret_cast<float*>(bs + (long)dy_pad * ldt);
    const int k8 = k_pad / 8;
    const int n16 = dy_pad * k8;  // 16-byte chunks of the staged B
    // eight chunks per thread in flight: all loads of a batch before its LDS stores. A
    // chunk is read whole (j8 + 8 <= k_pad <= ldb: inside the padded row), so that no load
    // waits for another; the entries of a row's last chunk past r are cleared on the store
    // side.
    constexpr int SBATCH = 8;
    for (int base = 0; base < n16; base += SBATCH * HES_TPB) {
        uint4 v[SBATCH];
#pragma unroll
        for (int u = 0; u < SBATCH; ++u) {
            const int e2 = base + u * HES_TPB + tid;
            v[u] = make_uint4(0u, 0u, 0u, 0u);
            const int i = e2 / k8, j8 = 8 * (e2 - i * k8);
            if (e2 < n16 && i < dy) v[u] = *reinterpret_cast<const uint4*>(Bc + (long)i * ldb + j8);
        }
#pragma unroll
        for (int u = 0; u < SBATCH; ++u) {
            const int e2 = base + u * HES_TPB + tid;
            const int i = e2 / k8, j8 = 8 * (e2 - i * k8);
            if (j8 + 8 > r) {
                uint32_t w4[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (j8 + 2 * q >= r) w4[q] = 0u;
                    else if (j8 + 2 * q + 1 >= r) w4[q] &= 0xFFFFu;  // the low half is entry j8 + 2q
                }
                v[u] = make_uint4(w4[0], w4[1], w4[2], w4[3]);
            }
            if (e2 < n16) *reinterpret_cast<uint4*>(bs + (long)i * ldt + j8) = v[u];
        }
    }
    residual_into(c, dy, f, y_rows, winv_rows, rows, es, red, phi);  // ends with a barrier
    for (int j = tid; j < r; j += HES_TPB) {
        double acc = 0.0;
#pragma unroll 4
        for (int i = 0; i < dy; ++i) acc += (double)__bfloat162float(bs[(long)i * ldt + j]) * (double)es[i];
        g[(long)c * r + j] = acc;
    }
    // lower blocks of B B^T: wave w takes blocks w, w + 4, w + 8 (at most 3 of the 10 at 4 row blocks)
    const int nl = lane & 31, h = lane >> 5;
    const int nmb = dy_pad / 32, nkc = k_pad / 16;
    const int nblocks = nmb * (nmb + 1) / 2;
    constexpr int MAXB = 3;
    f32x16 acc[MAXB];
    int bi_of[MAXB], bk_of[MAXB];
#pragma unroll
    for (int u = 0; u < MAXB; ++u) {
        const int bidx = wave + 4 * u;
        bi_of[u] = -1;
        bk_of[u] = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[u][j] = 0.f;
        if (bidx < nblocks) {
            int bi = 0;
            while ((bi + 1) * (bi + 2) / 2 <= bidx) ++bi;
            const int bk = bidx - bi * (bi + 1) / 2;
            bi_of[u] = bi;
            bk_of[u] = bk;
            for (int kc = 0; kc < nkc; ++kc) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(bs + (long)(32 * bi + nl) * ldt + 16 * kc + 8 * h);
                const bf16x8 b = *reinterpret_cast<const bf16x8*>(bs + (long)(32 * bk + nl) * ldt + 16 * kc + 8 * h);
                acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[u], 0, 0, 0);
            }
        }
    }
    __syncthreads();  // every wave has read B
    float* K = reinterpret_cast<float*>(bs);  // dy x (dy + 1), lower triangle
    const int ldk = dy + 1;
#pragma unroll
    for (int u = 0; u < MAXB; ++u) {
        if (bi_of[u] < 0) continue;
        const int colk = 32 * bk_of[u] + nl;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int row = 32 * bi_of[u] + 8 * (j >> 2) + 4 * h + (j & 3);
            if (row < dy && colk <= row) K[row * ldk + colk] = acc[u][j];
        }
    }
    __syncthreads();
    double* a = A + (long)c * strideA + (slot ? (long)(slot[c] ^ slot_xor) * slot_stride : 0);
    // with dinv: the diagonal blocks, 32 x 32 each, column-major, over K once the first wave
    // has read K into registers
    double* Ld = reinterpret_cast<double*>(bs);
    const int nfull = dy / 32;
    if (wave == 0) {  // the factorisation runs on the first wave alone (wavefront-scope steps)
        const int gg = lane >> 3, q = lane & 7;
        double v[MB][MB];
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const int i = gg + 8 * m;
#pragma unroll
            for (int cc = 0; cc < MB; ++cc) {
                const int kk = q + 8 * cc;
                // the identity is added in FP64, as the separate Gram kernel writes it; the read
                // is unconditional (clamped index) so that the reads issue back to back
                const float kv = K[min(i, dy - 1) * ldk + min(kk, dy - 1)];
                v[m][cc] = (cc <= m && i < dy && kk <= i) ? (double)kv + (i == kk ? 1.0 : 0.0) : 0.0;
            }
        }
        bool bad = false;
        if (q == 0) {  // column 0
#pragma unroll
            for (int m = 0; m < MB; ++m) col[gg + 8 * m] = v[m][0];
        }
        chol_sync<true>();
        double pivot = lane_value(v[0][0], 0);
        CholWavePhases<MB, 0, true>::run(v, col, pivs, dy, gg, q, bad, pivot,
                                         DiagBlockPublish<MB>{Ld, dready, dinv ? dy : 0, gg, q});
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const int i = gg + 8 * m;
#pragma unroll
            for (int cc = 0; cc <= m; ++cc) {
                const int kk = q + 8 * cc;
                // the lane's upper-triangle entries of a diagonal block pair are written as
                // zeros (with dinv they are left to the inverted blocks)
                if (i < dy && kk < dy && (kk <= i || !dinv)) a[(long)i * dy + kk] = (kk <= i) ? v[m][cc] : 0.0;
                if (dinv && nfull * 32 < dy && i < dy && kk <= i && (i >> 5) == nfull && (kk >> 5) == nfull)
                    Ld[nfull * 1024 + (kk & 31) * 32 + (i & 31)] = v[m][cc];
            }
        }
        chol_sync<true>();
        double ls = 0.0;
        for (int j = lane; j < dy; j += 64) ls += log(pivs[j]);
        for (int o = 32; o > 0; o >>= 1) ls += __shfl_xor(ls, o);
        const bool any_bad = __any(bad);
        if (lane == 0) {
            if (logdet) logdet[c] = 0.5 * ls;
            if (ok) ok[c] = any_bad ? 0 : 1;
        }
        if (dinv && nfull * 32 < dy) {  // the short last block
            const int nb = dy - 32 * nfull;
            if (nb <= 8) invert_diag_block<8>(Ld + nfull * 1024, nb, lane, a, dy, 32 * nfull);
            else invert_diag_block<32>(Ld + nfull * 1024, nb, lane, a, dy, 32 * nfull);
        }
    } else if (dinv && wave - 1 < nfull) {
        const int b = wave - 1;
        // wait for the first wave to publish block b (bounded: a lost flag cannot hang the
        // launch; the factorisation always reaches it)
        for (int spins = 0; spins < (1 << 22); ++spins) {
            if (__hip_atomic_load(dready + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
            __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        invert_diag_block<32>(Ld + b * 1024, 32, lane, a, dy, 32 * b);
    }
}

// Fused Gram + factor of the dual form on the mixed path: d_y <= 104 and the staged B
// within LDS (two blocks per CU when it takes at most ~78 KB).
static size_t gram_chol_lds(int r, int dy) {
    const size_t dy_pad = (dy + 31) / 32 * 32, k_pad = (r + 15) / 16 * 16, ldt = k_pad + 8;
    const size_t b = dy_pad * ldt * sizeof(__hip_bfloat16) + (size_t)dy * sizeof(float);
    const size_t k = (size_t)dy * (dy + 1) * sizeof(float);
    const size_t d = (dy_pad / 32) * 1024 * sizeof(double);  // the diagonal blocks (dinv)
    return std::max(std::max(b, k), d);
}

bool gram_chol_bf16_fits(int r, int dy) { return dy <= 104 && gram_chol_lds(r, dy) <= 160 * 1024 - 4096; }

void launch_gram_chol_bf16(dino_problem* p, int n, const __hip_bfloat16* B, const float* f, double* phi, double* A,
                           long strideA, const int32_t* slot, int slot_xor, long slot_stride, double* g,
                           double* logdet, int32_t* ok, int dinv, hipStream_t st) {
    const int r = p->r, dy = p->d_y;
    DINO_REQUIRE(gram_chol_bf16_fits(r, dy), DINO_EINVAL, "d_y x r beyond the fused Gram + factor kernel");
    const int dy_pad = (dy + 31) / 32 * 32;
    const int k_pad = (r + 15) / 16 * 16;
    const int ldt = k_pad + 8;
    const size_t lds = gram_chol_lds(r, dy);
    static bool attr = false;
    if (!attr) {
        DINO_HIP(hipFuncSetAttribute((const void*)gram_chol_bf16_kernel<13>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     160 * 1024 - 4096));
        attr = true;
    }
    hipLaunchKernelGGL(gram_chol_bf16_kernel<13>, dim3(n), dim3(HES_TPB), lds, st, dy, r, (r + 31) / 32 * 32, dy_pad,
                       k_pad, ldt, B, f, p->y, p->winv, p->meta.row, phi, A, strideA, slot, slot_xor, slot_stride, g,
                       logdet, ok, dinv);
    DINO_HIP(hipGetLastError());
}

// LDS of hess_bf16_kernel: B^T (r_pad x (dy_pad + 8) BF16) and the residual (dy floats).
static size_t hess_bf16_lds(int r, int dy) {
    const size_t dy_pad = (dy + 15) / 16 * 16, r_pad = (r + 31) / 32 * 32;
    return r_pad * (dy_pad + 8) * sizeof(__hip_bfloat16) + (size_t)dy * sizeof(float);
}

bool hess_bf16_lds_fits(int r, int dy) { return hess_bf16_lds(r, dy) <= 160 * 1024 - 64; }

void launch_hess_bf16(dino_problem* p, int n, const __hip_bfloat16* B, const float* f, double* phi, double* A,
                      long strideA, const int32_t* slot, int slot_xor, long slot_stride, double* g, hipStream_t st) {
    const int r = p->r, dy = p->d_y;
    const int dy_pad = (dy + 15) / 16 * 16;
    const int ldt = dy_pad + 8;  // 16-byte aligned rows, shifted banks
    const int r_pad = (r + 31) / 32 * 32;
    const size_t lds = hess_bf16_lds(r, dy);
    if (lds > 160 * 1024 - 64 || tuned_choice(TUNE_HESS, r, dy, 0) == 1) {
        DINO_REQUIRE(dy <= 1024, DINO_EINVAL, "d_y above 1024");
        const int T = (r + 63) / 64, ntile = T * (T + 1) / 2;
        const long total = (long)n * ntile, blocks = (total + 7) / 8 * 8;
        DINO_REQUIRE(blocks < (1L << 31), DINO_EINVAL, "too many Hessian tiles for one launch");
        if (n > 0)
            hipLaunchKernelGGL(hess_bf16_tiled_kernel, dim3((unsigned)blocks), dim3(HES_TPB), 0, st, n, dy, r, r_pad,
                               ntile, B, f, p->y, p->winv, p->meta.row, phi, A, strideA, slot, slot_xor, slot_stride,
                               g);
        DINO_HIP(hipGetLastError());
        return;
    }
    static bool attr = false;
    if (!attr) {
        DINO_HIP(hipFuncSetAttribute((const void*)hess_bf16_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     160 * 1024 - 64));
        attr = true;
    }
    hipLaunchKernelGGL(hess_bf16_kernel, dim3(n), dim3(HES_TPB), lds, st, dy, r, r_pad, dy_pad, ldt, B, f, p->y,
                       p->winv, p->meta.row, phi, A, strideA, slot, slot_xor, slot_stride, g);
    DINO_HIP(hipGetLastError());
}

void launch_to_float(long count, const double* x, float* xf, hipStream_t st) {
    const int blocks = (int)std::min<long>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(to_float_kernel, dim3(blocks), dim3(256), 0, st, count, x, xf);
    DINO_HIP(hipGetLastError());
}

// H[c][j][k] = A[c][max(j,k)][min(j,k)] - [j == k]: the full H from the lower I + H.
__global__ void sym_from_lower_kernel(int n, int r, const double* __restrict__ A, double* __restrict__ H) {
    const long rr = (long)r * r, total = (long)n * rr;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const long c = e / rr;
        const int j = (int)((e % rr) / r), k = (int)(e % r);
        const int hi = j > k ? j : k, lo = j > k ? k : j;
        H[e] = A[c * rr + (long)hi * r + lo] - (j == k ? 1.0 : 0.0);
    }
}

void launch_sym_from_lower(int n, int r, const double* A, double* H, hipStream_t st) {
    const long total = (long)n * r * r;
    const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(sym_from_lower_kernel, dim3(blocks), dim3(256), 0, st, n, r, A, H);
    DINO_HIP(hipGetLastError());
}

void launch_to_double(long count, const float* xf, double* x, hipStream_t st) {
    const int blocks = (int)std::min<long>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(to_double_kernel, dim3(blocks), dim3(256), 0, st, count, xf, x);
    DINO_HIP(hipGetLastError());
}


}  // namespace dino
