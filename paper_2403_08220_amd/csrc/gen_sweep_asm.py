"""Writes sweep_asm.inc: one layer of the width-416 BF16 reduced-Jacobian sweep (13
output row blocks of 32 x 26 K chunks of 16) as a single inline-asm block for gfx950.

Register roles: the 13 accumulators (Lambda^T, FP32, 16 VGPRs each) are pinned to
v0..v207 and the 26 B operands (bf16(d * Lambda), one per K chunk, 4 AGPRs each) to
a0..a103, so that the block can address single elements of both; a ring of 6 A-operand
sets (1 KB weight tiles read from LDS, one ds_read_b128 per lane) is in AGPRs.

Per work item j (output row block) of the layer, when j < n:
  * if the item three ahead exists (j < T): copy its tiles into the ring buffer freed by
    item j - 1 (seven global_load_lds_dwordx4 per wave, M0 = LDS destination, one after
    every third MFMA of the item);
  * (block start, if df != 0) copy the next layer's gelu' rows of the wave's chains into
    the wave's LDS region (four copies, complete when the block ends);
  * 26 MFMAs v_mfma_f32_32x32x16_bf16 into accumulator j (the first one starts from 0
    for a layer without the residual term), their A operands read 5 ahead;
  * after the last read of the item: drain the reads, wait until item j + 1 is resident
    for every wave (vmcnt + s_barrier; all waves are then done reading item j - 1's
    buffer, which the next copy overwrites), then issue the first reads of item j + 1,
    which overlap the last MFMAs of item j.
Items j >= n are skipped and their accumulators set to zero (one MFMA with zero
operands).

Next layer's B operands (ff != 0: all 13 items run and the gelu' rows of the next layer
are in the wave's LDS region): during the last item, chunk k of the next layer,
bf16(d_next * Lambda rows 16k..16k+15), is formed once the last MFMA reading the
current operand k has issued two MFMAs earlier (k < 24; rows of accumulators 0..11,
which are final); chunks 24 and 25 (accumulator 12) follow the last MFMA. Each chunk:
two ds_read_b128 of gelu' values (issued one MFMA ahead, two register sets), eight
v_mul_f32, four v_cvt_pk_bf16_f32 and four v_accvgpr_write into the operand's AGPRs.
The arithmetic and rounding equal the compiler's formation between blocks.

Every LDS read is waited for inside the block (s_waitcnt lgkmcnt counted over all reads
in flight; LDS reads return in order); the block ends with wait states that cover the
last MFMA's write of an accumulator before vector instructions read it.
Run: python gen_sweep_asm.py
"""
import os

D = 5          # reads ahead of the MFMA chain
RING = 6       # register sets in the ring
NKC = 26       # K chunks (MFMAs) per item
NITEMS = 13    # output row blocks per layer
ITEM_BYTES = 28 * 1024   # tiles per item (28) x 1 KB
NQ = 7         # tile copies per wave per item
COPY_EVERY = 3  # one copy after every third MFMA of the item (all before its boundary)
TD = 240       # gelu' values of two chunks: v[240:247], v[248:255]
TC = 236       # converted pairs: v[236:239]


def line(s):
    return f'        "{s}\\n\\t"'


def label(s):
    return f'        "{s}:\\n\\t"'


class Reads:
    """LDS reads in flight since the last full drain, in issue order (they complete in order)."""

    def __init__(self):
        self.q = []

    def issue(self, tag):
        self.q.append(tag)

    def drain(self):
        self.q = []

    def wait(self, tag):
        # wait until `tag` has completed: at most the reads issued after it stay in flight
        if tag not in self.q:
            return []
        i = self.q.index(tag)
        n = len(self.q) - 1 - i
        assert n <= 15
        self.q = self.q[i + 1:]
        return [line(f"s_waitcnt lgkmcnt({n})")]

    def copy(self):
        r = Reads()
        r.q = list(self.q)
        return r


def layer():
    total = NITEMS * NKC
    addr = lambda j: "%[va]" if j % 2 == 0 else "%[vb]"

    def rd(c, reads):
        reads.issue(("r", c))
        return line(f"ds_read_b128 %[t{c % RING}], {addr(c // NKC)} offset:{(c % NKC) * 1024}")

    def stage_setup(j):
        # copies of item j + 3 (if it exists) go to the ring buffer before the current one
        # (ring of 4): LDS destination st and global source s[60:61] of this wave's first tile
        return [line(f"s_cmp_lt_i32 {j}, %[tl]"),
                line("s_cbranch_scc0 1f"),
                line("s_sub_u32 %[st], %[sc], " + str(ITEM_BYTES)),
                line("s_cmp_eq_u32 %[sc], %[sb]"),
                line("s_cselect_b32 %[st], %[sz], %[st]"),
                line("s_add_u32 %[st], %[st], %[sw]"),
                line("s_add_u32 s60, %[sl], %[so]"),
                line("s_addc_u32 s61, %[sh], 0"),
                line("s_add_u32 s60, s60, %[sw]"),
                line("s_addc_u32 s61, s61, 0"),
                line("s_add_u32 %[so], %[so], " + str(ITEM_BYTES)),
                label("1")]

    def stage_copy(j, q):
        # tile copy q of this wave for item j + 3; the seven copies are spread over the
        # item's first MFMAs (copies issued back to back slow the LDS reads beside them)
        s = [line(f"s_cmp_lt_i32 {j}, %[tl]"),
             line("s_cbranch_scc0 1f")]
        if q > 0:
            s.append(line("s_add_u32 s60, s60, 4096"))
            s.append(line("s_addc_u32 s61, s61, 0"))
        s.append(line("s_mov_b32 m0, %[st]") if q == 0 else line(f"s_add_u32 m0, %[st], {q * 4096}"))
        s.append(line("s_nop 0"))  # one wait state between an SALU write of M0 and an LDS DMA
        s.append(line("global_load_lds_dwordx4 %[vl], s[60:61]"))
        s.append(label("1"))
        return s

    def boundary(j, reads):
        # item j + 1 resident for all waves; ring buffer and read address of item j + 1.
        # The copies younger than item j + 1 are those of items j + 2 and j + 3 and, for
        # j < 2, the four gelu' row copies issued at the start of the block.
        extra = [line("s_cmp_eq_u32 %[df], 0"), line("s_cbranch_scc1 7f"), line("s_waitcnt vmcnt(18)"),
                 line("s_branch 5f"), label("7")] if j < 2 else []
        reads.drain()
        return [line("s_waitcnt lgkmcnt(0)"),
                line(f"s_cmp_lt_i32 {j}, %[tl]"),
                line("s_cbranch_scc0 4f")] + extra + [
                line("s_waitcnt vmcnt(14)"),
                line("s_branch 5f"),
                label("4"),
                line("s_waitcnt vmcnt(0)"),
                label("5"),
                line("s_barrier"),
                line("s_add_u32 %[sc], %[sc], " + str(ITEM_BYTES)),
                line("s_cmp_eq_u32 %[sc], %[se]"),
                line("s_cselect_b32 %[sc], %[sb], %[sc]"),
                line(f"v_add_u32 {addr(j + 1)}, %[sc], %[vl]")]

    def d_reads(k, reads):
        # gelu' values of next-layer chunk k: rows 16k + 4h + 0..3 and 16k + 8 + 4h + 0..3
        t = TD + 8 * (k % 2)
        reads.issue(("d", k, 0))
        reads.issue(("d", k, 1))
        return [line(f"ds_read_b128 v[{t}:{t + 3}], %[vd] offset:{64 * k}"),
                line(f"ds_read_b128 v[{t + 4}:{t + 7}], %[vd] offset:{64 * k + 32}")]

    def form(k, reads):
        # operand k of the next layer = bf16(d * Lambda[16k .. 16k + 15]) in a[4k : 4k + 3]
        t = TD + 8 * (k % 2)
        lam0 = 16 * (k // 2) + 8 * (k % 2)
        s = reads.wait(("d", k, 1))
        for jj in range(8):
            s.append(line(f"v_mul_f32 v{t + jj}, v{lam0 + jj}, v{t + jj}"))
        for p in range(4):
            s.append(line(f"v_cvt_pk_bf16_f32 v{TC + p}, v{t + 2 * p}, v{t + 2 * p + 1}"))
        for p in range(4):
            s.append(line(f"v_accvgpr_write_b32 a{4 * k + p}, v{TC + p}"))
        return s

    def item(j, reads, fused):
        s = stage_setup(j)
        for kc in range(NKC):
            c = j * NKC + kc
            mf = lambda src: line(f"v_mfma_f32_32x32x16_bf16 %[l{j}], %[t{c % RING}], %[b{kc}], {src}")
            s += reads.wait(("r", c))
            if kc == 0:
                s += [line("s_bitcmp1_b32 %[n], 8"), line("s_cbranch_scc0 2f"), mf("0"), line("s_branch 3f"),
                      label("2"), mf(f"%[l{j}]"), label("3")]
            else:
                s.append(mf(f"%[l{j}]"))
            if kc % COPY_EVERY == 0 and kc // COPY_EVERY < NQ:
                s += stage_copy(j, kc // COPY_EVERY)
            if kc == NKC - D:
                s += boundary(j, reads)
            if c + D < total:
                s.append(rd(c + D, reads))
            if fused:
                if 1 <= kc <= NKC - 1:
                    s += d_reads(kc - 1, reads)
                if kc >= 2:
                    s += form(kc - 2, reads)
        if fused:
            s += d_reads(NKC - 1, reads)
            # the last MFMA's accumulator (chunks 24 and 25) is read by vector instructions
            s += [line("s_nop 7"), line("s_nop 7"), line("s_nop 4")]
            s += form(NKC - 2, reads)
            s += form(NKC - 1, reads)
        return s

    out = []
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
    out.append(label("6"))
    out.append(line("v_add_u32 %[va], %[sc], %[vl]"))
    reads = Reads()
    for c in range(D):
        out.append(rd(c, reads))
    last = NITEMS - 1
    fused_reads = None
    for j in range(NITEMS):
        out.append(line(f"s_cmp_le_u32 %[nn], {j}"))
        out.append(line(f"s_cbranch_scc1 {100 + j}f"))
        if j == last:
            fused_reads = reads.copy()
            out += [line("s_cmp_eq_u32 %[ff], 0"), line("s_cbranch_scc0 300f")]
        out += item(j, reads, False)
    out.append(line("s_branch 199f"))
    for j in range(NITEMS):
        out.append(label(str(100 + j)))
        out.append(line(f"v_mfma_f32_32x32x16_bf16 %[l{j}], %[z], %[z], 0"))
    out.append(line("s_branch 199f"))
    # the last item with the next layer's operand formation
    out.append(label("300"))
    out += item(last, fused_reads, True)
    out.append(label("199"))
    out.append(line("s_waitcnt lgkmcnt(0)"))
    # the gelu' row copies are complete (at most the last item's seven tile copies are younger)
    out.append(line("s_waitcnt vmcnt(7)"))
    out.append(line("s_mov_b32 m0, %[ms]"))
    out.append(line("s_nop 7"))
    out.append(line("s_nop 7"))
    out.append('        "s_nop 4"')
    body = "\n".join(out)
    lam = ", ".join(f'[l{i}] "+{{v[{16 * i}:{16 * i + 15}]}}"(lam[{i}])' for i in range(NITEMS))
    bops = ", ".join(f'[b{i}] "+{{a[{4 * i}:{4 * i + 3}]}}"(bop[{i}])' for i in range(NKC))
    ring = ", ".join(f'[t{i}] "=&a"(t{i})' for i in range(RING))
    temps = (f'[x0] "=&{{v[{TC}:{TC + 3}]}}"(x0), [x1] "=&{{v[{TD}:{TD + 3}]}}"(x1), '
             f'[x2] "=&{{v[{TD + 4}:{TD + 7}]}}"(x2), [x3] "=&{{v[{TD + 8}:{TD + 11}]}}"(x3), '
             f'[x4] "=&{{v[{TD + 12}:{TD + 15}]}}"(x4)')
    dins = ", ".join(f'[do{u}] "v"(doff[{u}])' for u in range(4))
    return f"""// n: bits 0-7 items of the layer (1..13), bit 8 set: the layer overwrites Lambda (no residual);
// tl: items j < tl have an item three ahead to copy and two younger items in flight;
// sc: LDS address of item 0's ring buffer; so: byte offset of the tiles of item 3;
// sl/sh: tile base address; sb/se/sz: ring start, end and last buffer; sw: wave * 1 KB;
// vl: lane * 16 (LDS read and tile copy offset of the lane); z: a zero operand;
// df != 0: copy 4 KB of gelu' rows, 16 B per lane at dsb + doff[u], to LDS dm + u KB;
// ff != 0 (requires df != 0 and n = 13): form the next layer's operands in bop from the
// gelu' row at LDS address vd (the lane's chain row + 16 h bytes).
__device__ __forceinline__ void sweep_layer13(f32x16 (&lam)[13], bf16x8 (&bop)[26], uint32_t n, int32_t tl, uint32_t sc, uint32_t so, uint32_t sl, uint32_t sh, uint32_t sb, uint32_t se, uint32_t sz,
        uint32_t sw, uint32_t vl, bf16x8 z, uint32_t df, uint64_t dsb, uint32_t dm,
        const uint32_t (&doff)[4], uint32_t ff, uint32_t vd) {{
    bf16x8 {", ".join(f"t{i}" for i in range(RING))};
    f32x4 x0, x1, x2, x3, x4;
    uint32_t va, vb, st, nn, ms;
    asm volatile(
{body}
        : {lam}, {bops}, {ring}, {temps},
          [va] "=&v"(va), [vb] "=&v"(vb), [st] "=&s"(st), [nn] "=&s"(nn), [ms] "=&s"(ms), [sc] "+s"(sc), [so] "+s"(so)
        : {dins}, [vl] "v"(vl), [vd] "v"(vd), [z] "a"(z), [n] "s"(n), [tl] "s"(tl), [sl] "s"(sl),
          [sh] "s"(sh), [sb] "s"(sb), [se] "s"(se), [sz] "s"(sz), [sw] "s"(sw), [df] "s"(df), [dsb] "s"(dsb),
          [dm] "s"(dm), [ff] "s"(ff)
        : "s60", "s61", "scc", "memory");
    // the ring registers and temporaries are consumed here (every read above has completed)
    asm volatile("" ::{", ".join(f'"a"(t{i})' for i in range(RING))}, "v"(va), "v"(vb), "v"(x0), "v"(x1), "v"(x2),
                 "v"(x3), "v"(x4));
}}
"""


def formation(src):
    """One layer's 26 B operands bf16(d * Lambda) outside the layer block, with the
    registers of the block: gelu' values from the wave's LDS region (src "lds": vd is the
    lane's LDS byte address) or from global memory (src "global": ga is the lane's 64-bit
    address), loaded one chunk ahead into two register sets and counted with lgkmcnt
    (LDS) or vmcnt (global: vector memory loads, the tile copies in flight included,
    complete in issue order, so the count over this block's loads is a sufficient wait)."""
    out = []
    cnt = "lgkmcnt" if src == "lds" else "vmcnt"

    def loads(k):
        t = TD + 8 * (k % 2)
        if src == "lds":
            return [line(f"ds_read_b128 v[{t}:{t + 3}], %[vd] offset:{64 * k}"),
                    line(f"ds_read_b128 v[{t + 4}:{t + 7}], %[vd] offset:{64 * k + 32}")]
        return [line(f"global_load_dwordx4 v[{t}:{t + 3}], %[ga], off offset:{64 * k}"),
                line(f"global_load_dwordx4 v[{t + 4}:{t + 7}], %[ga], off offset:{64 * k + 32}")]

    out += loads(0)
    for k in range(NKC):
        if k + 1 < NKC:
            out += loads(k + 1)
        out.append(line(f"s_waitcnt {cnt}({2 if k + 1 < NKC else 0})"))
        t = TD + 8 * (k % 2)
        lam0 = 16 * (k // 2) + 8 * (k % 2)
        for jj in range(8):
            out.append(line(f"v_mul_f32 v{t + jj}, v{lam0 + jj}, v{t + jj}"))
        for p in range(4):
            out.append(line(f"v_cvt_pk_bf16_f32 v{TC + p}, v{t + 2 * p}, v{t + 2 * p + 1}"))
        for p in range(4):
            out.append(line(f"v_accvgpr_write_b32 a{4 * k + p}, v{TC + p}"))
    out[-1] = out[-1].replace('\\n\\t"', '"')
    body = "\n".join(out)
    lam = ", ".join(f'"{{v[{16 * i}:{16 * i + 15}]}}"(lam[{i}])' for i in range(NITEMS))
    bops = ", ".join(f'"={{a[{4 * i}:{4 * i + 3}]}}"(bop[{i}])' for i in range(NKC))
    temps = (f'"=&{{v[{TC}:{TC + 3}]}}"(x0), "=&{{v[{TD}:{TD + 3}]}}"(x1), "=&{{v[{TD + 4}:{TD + 7}]}}"(x2), '
             f'"=&{{v[{TD + 8}:{TD + 11}]}}"(x3), "=&{{v[{TD + 12}:{TD + 15}]}}"(x4)')
    name, arg, op = (("sweep_form13_lds", "uint32_t vd", '[vd] "v"(vd)') if src == "lds" else
                     ("sweep_form13_global", "const float* ga", '[ga] "v"(ga)'))
    return f"""
// The B operands of one layer from gelu' rows in {"the wave's LDS region (vd: LDS byte address of the lane's row + 16 h)" if src == "lds" else "global memory (ga: the lane's row + 4 h floats)"}.
__device__ __forceinline__ void {name}(const f32x16 (&lam)[13], bf16x8 (&bop)[26], {arg}) {{
    f32x4 x0, x1, x2, x3, x4;
    asm volatile(
{body}
        : {bops}, {temps}
        : {lam}, {op}
        : "memory");
    asm volatile("" ::"v"(x0), "v"(x1), "v"(x2), "v"(x3), "v"(x4));
}}
"""


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    text = ("// Generated by gen_sweep_asm.py: one layer of the width-416 BF16 sweep as an inline-asm block.\n"
            "// Included by kernels_mfma.hip inside namespace dino (bf16x8 / f32x16 / f32x4 defined there).\n\n"
            + layer() + formation("lds") + formation("global"))
    with open(os.path.join(here, "sweep_asm.inc"), "w") as f:
        f.write(text)


if __name__ == "__main__":
    main()
