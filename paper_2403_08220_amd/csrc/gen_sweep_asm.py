"""Writes sweep_asm.inc: one layer of the width-416 BF16 reduced-Jacobian sweep (13
output row blocks of 32 x 26 K chunks of 16) as a single inline-asm block for gfx950.

Register roles: the 13 accumulators (Lambda^T, FP32, 16 VGPRs each) are in VGPRs; the
26 B operands (bf16(d * Lambda), one per K chunk) and a ring of 6 A-operand sets (1 KB
weight tiles read from LDS, one ds_read_b128 per lane) are in AGPRs.

Per work item j (output row block) of the layer, when j < n:
  * if the item three ahead exists (j < T): copy its tiles into the ring buffer freed by
    item j - 1 (seven global_load_lds_dwordx4 per wave, M0 = LDS destination);
  * (block start, if df != 0) copy the next layer's gelu' rows of the wave's chains into
    the wave's LDS region (four copies, complete when the block ends);
  * 26 MFMAs v_mfma_f32_32x32x16_bf16 into accumulator j (the first one starts from 0
    for a layer without the residual term), their A operands read 5 ahead;
  * after the last read of the item: drain the reads, wait until item j + 1 is resident
    for every wave (vmcnt + s_barrier; all waves are then done reading item j - 1's
    buffer, which the next copy overwrites), then issue the first reads of item j + 1,
    which overlap the last MFMAs of item j.
Items j >= n are skipped and their accumulators set to zero (one MFMA with zero
operands). Every LDS read is waited for inside the block (s_waitcnt lgkmcnt; LDS reads
return in order); the block ends with wait states that cover the last MFMA's write of
an accumulator before vector instructions read it. Run: python gen_sweep_asm.py
"""
import os

D = 5          # reads ahead of the MFMA chain
RING = 6       # register sets in the ring
NKC = 26       # K chunks (MFMAs) per item
NITEMS = 13    # output row blocks per layer
ITEM_BYTES = 28 * 1024   # tiles per item (28) x 1 KB
NQ = 7         # tile copies per wave per item


def line(s):
    return f'        "{s}\\n\\t"'


def layer():
    total = NITEMS * NKC
    addr = lambda j: "%[va]" if j % 2 == 0 else "%[vb]"
    rd = lambda c: line(f"ds_read_b128 %[t{c % RING}], {addr(c // NKC)} offset:{(c % NKC) * 1024}")
    out = []

    def stage(j):
        # copy item j + 3 into the buffer before the current one (ring of 4), if it exists
        s = [line(f"s_cmp_lt_i32 {j}, %[tl]"),
             line("s_cbranch_scc0 1f"),
             line("s_sub_u32 %[st], %[sc], " + str(ITEM_BYTES)),
             line("s_cmp_eq_u32 %[sc], %[sb]"),
             line("s_cselect_b32 %[st], %[sz], %[st]"),
             line("s_add_u32 %[st], %[st], %[sw]"),
             line("s_add_u32 s60, %[sl], %[so]"),
             line("s_addc_u32 s61, %[sh], 0"),
             line("s_add_u32 s60, s60, %[sw]"),
             line("s_addc_u32 s61, s61, 0")]
        for q in range(NQ):
            if q > 0:
                s.append(line("s_add_u32 s60, s60, 4096"))
                s.append(line("s_addc_u32 s61, s61, 0"))
            s.append(line("s_mov_b32 m0, %[st]") if q == 0 else line(f"s_add_u32 m0, %[st], {q * 4096}"))
            s.append(line("s_nop 0"))  # one wait state between an SALU write of M0 and an LDS DMA
            s.append(line("global_load_lds_dwordx4 %[vl], s[60:61]"))
        s.append(line("s_add_u32 %[so], %[so], " + str(ITEM_BYTES)))
        s.append('        "1:\\n\\t"')
        return s

    def boundary(j):
        # item j + 1 resident for all waves; ring buffer and read address of item j + 1.
        # The copies younger than item j + 1 are those of items j + 2 and j + 3 and, for
        # j < 2, the four gelu' row copies issued at the start of the block.
        extra = [line("s_cmp_eq_u32 %[df], 0"), line("s_cbranch_scc1 7f"), line("s_waitcnt vmcnt(18)"),
                 line("s_branch 5f"), '        "7:\\n\\t"'] if j < 2 else []
        return [line("s_waitcnt lgkmcnt(0)"),
                line(f"s_cmp_lt_i32 {j}, %[tl]"),
                line("s_cbranch_scc0 4f")] + extra + [
                line("s_waitcnt vmcnt(14)"),
                line("s_branch 5f"),
                '        "4:\\n\\t"',
                line("s_waitcnt vmcnt(0)"),
                '        "5:\\n\\t"',
                line("s_barrier"),
                line("s_add_u32 %[sc], %[sc], " + str(ITEM_BYTES)),
                line("s_cmp_eq_u32 %[sc], %[se]"),
                line("s_cselect_b32 %[sc], %[sb], %[sc]"),
                line(f"v_add_u32 {addr(j + 1)}, %[sc], %[vl]")]

    # M0 is reserved (the compiler does not honour it as a clobber): saved here, restored at the end
    out.append(line("s_mov_b32 %[ms], m0"))
    out.append(line("s_waitcnt lgkmcnt(0)"))
    out.append(line("s_and_b32 %[nn], %[n], 0xff"))
    # gelu' rows of the next layer (two chain rows, 4 KB) into the wave's LDS region, if df
    out += [line("s_cmp_eq_u32 %[df], 0"), line("s_cbranch_scc1 6f")]
    for u in range(4):
        out.append(line("s_mov_b32 m0, %[dm]") if u == 0 else line(f"s_add_u32 m0, %[dm], {u * 1024}"))
        out.append(line("s_nop 0"))
        out.append(line(f"global_load_lds_dwordx4 %[do{u}], %[dsb]"))
    out.append('        "6:\\n\\t"')
    out.append(line("v_add_u32 %[va], %[sc], %[vl]"))
    for c in range(D):
        out.append(rd(c))
    issued = D
    for c in range(total):
        j, kc = divmod(c, NKC)
        if kc == 0:
            out.append(line(f"s_cmp_le_u32 %[nn], {j}"))
            out.append(line(f"s_cbranch_scc1 {100 + j}f"))
            out += stage(j)
        mf = lambda src: line(f"v_mfma_f32_32x32x16_bf16 %[l{j}], %[t{c % RING}], %[b{kc}], {src}")
        if kc <= NKC - D:
            out.append(line(f"s_waitcnt lgkmcnt({issued - 1 - c})"))
        if kc == 0:
            out += [line("s_bitcmp1_b32 %[n], 8"), line("s_cbranch_scc0 2f"), mf("0"), line("s_branch 3f"),
                    '        "2:\\n\\t"', mf(f"%[l{j}]"), '        "3:\\n\\t"']
        else:
            out.append(mf(f"%[l{j}]"))
        if kc == NKC - D:
            out += boundary(j)
        if c + D < total:
            out.append(rd(c + D))
            issued += 1
    out.append(line("s_branch 199f"))
    for j in range(NITEMS):
        out.append(f'        "{100 + j}:\\n\\t"')
        out.append(line(f"v_mfma_f32_32x32x16_bf16 %[l{j}], %[z], %[z], 0"))
    out.append('        "199:\\n\\t"')
    out.append(line("s_waitcnt lgkmcnt(0)"))
    # the gelu' row copies are complete (at most the last item's seven tile copies are younger)
    out.append(line("s_waitcnt vmcnt(7)"))
    out.append(line("s_mov_b32 m0, %[ms]"))
    out.append(line("s_nop 7"))
    out.append(line("s_nop 7"))
    out.append('        "s_nop 4"')
    body = "\n".join(out)
    lam = ", ".join(f'[l{i}] "+v"(lam[{i}])' for i in range(NITEMS))
    ring = ", ".join(f'[t{i}] "=&a"(t{i})' for i in range(RING))
    bins = ", ".join(f'[b{i}] "a"(bop[{i}])' for i in range(NKC))
    dins = ", ".join(f'[do{u}] "v"(doff[{u}])' for u in range(4))
    return f"""// n: bits 0-7 items of the layer (1..13), bit 8 set: the layer overwrites Lambda (no residual);
// tl: items j < tl have an item three ahead to copy and two younger items in flight;
// sc: LDS address of item 0's ring buffer; so: byte offset of the tiles of item 3;
// sl/sh: tile base address; sb/se/sz: ring start, end and last buffer; sw: wave * 1 KB;
// vl: lane * 16 (LDS read and tile copy offset of the lane); z: a zero operand;
// df != 0: copy 4 KB of gelu' rows, 16 B per lane at dsb + doff[u], to LDS dm + u KB.
__device__ __forceinline__ void sweep_layer13(f32x16 (&lam)[13], const bf16x8 (&bop)[26], uint32_t n, int32_t tl, uint32_t sc, uint32_t so, uint32_t sl, uint32_t sh, uint32_t sb, uint32_t se, uint32_t sz,
        uint32_t sw, uint32_t vl, bf16x8 z, uint32_t df, uint64_t dsb, uint32_t dm,
        const uint32_t (&doff)[4]) {{
    bf16x8 {", ".join(f"t{i}" for i in range(RING))};
    uint32_t va, vb, st, nn, ms;
    asm volatile(
{body}
        : {lam}, {ring}, [va] "=&v"(va), [vb] "=&v"(vb), [st] "=&s"(st), [nn] "=&s"(nn), [ms] "=&s"(ms), [sc] "+s"(sc), [so] "+s"(so)
        : {bins}, {dins}, [vl] "v"(vl), [z] "a"(z), [n] "s"(n), [tl] "s"(tl), [sl] "s"(sl),
          [sh] "s"(sh), [sb] "s"(sb), [se] "s"(se), [sz] "s"(sz), [sw] "s"(sw), [df] "s"(df), [dsb] "s"(dsb),
          [dm] "s"(dm)
        : "s60", "s61", "scc", "memory");
    // the ring registers are consumed here (every read above has completed)
    asm volatile("" ::{", ".join(f'"a"(t{i})' for i in range(RING))}, "v"(va), "v"(vb));
}}
"""


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    text = ("// Generated by gen_sweep_asm.py: one layer of the width-416 BF16 sweep as an inline-asm block.\n"
            "// Included by kernels_mfma.hip inside namespace dino (bf16x8 / f32x16 defined there).\n\n"
            + layer())
    with open(os.path.join(here, "sweep_asm.inc"), "w") as f:
        f.write(text)


if __name__ == "__main__":
    main()
