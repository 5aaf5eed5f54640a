"""Writes xd_wchain_asm.h: the register chain of the wide tiers as gfx950
assembly, one function per (registers C, parity).

The chain updates the registers of a band's span in one fall-through run of
identical blocks: upwards from rlo on even anti-diagonals (neighbour slot s-1:
a wave_ror rotation, lane 0 from the register walked before), downwards from
rhi on odd ones (slot s+1: wave_rol, lane 63 from the register walked
before).  Each block is the cell update of one register in the gap-free W
form with narrow two-bit score fields:

    rotate the previous anti-diagonal's register       v_mov_b32_dpp
    score field                                         v_bfe_u32
    neighbour lane from the register walked before      v_cndmask_b32
    diagonal term W(d-2) + s + 2|gap|                   v_add3_u32
    the recurrence                                      v_max3_i32
    X-drop test                                         v_cmp
    end of the span?                                    s_cmp, s_cbranch
    -inf for pruned cells                               v_cndmask
    running maximum for the improvement test            v_max_i32

The span's two edge registers are also clipped to the computed range: a
table of branches enters the chain at a head block, which ands the X-drop
test with the entry register's lane mask and keeps the result (its
survivors); the block that ends the chain leaves through a tail that ands
the test with the last register's mask.  So cells outside the range come out
-inf, the running maximum sees only surviving cells of the range, and both
edge registers' survivor masks come back without another pass.

The rotation of each block alternates between two registers, so the block
after it finds it as its neighbour without a copy.

WFirst<C>::run is the search for the first (lowest) slot of the span whose
cell exceeds a value, used when best can rise by exactly one: a table of
branches enters at the span's lowest register, and each register is one
compare and two branches.

Run from the repository root: python paper_2002_05200_amd/csrc/gen_wchain.py
"""
import os

CS = (2, 4, 8, 16, 32)
HERE = os.path.dirname(os.path.abspath(__file__))


def _reg(C, par, k):
    """Register at chain position k."""
    return k if par == 0 else C - 1 - k


def _cell(C, par, k):
    """The cell update up to the X-drop test (VCC = survivors before clipping)."""
    r = _reg(C, par, k)
    own, carry = ("tA", "tB") if k % 2 == 0 else ("tB", "tA")
    rot = "wave_ror:1" if par == 0 else "wave_rol:1"
    return [
        f'"v_mov_b32_dpp %[{own}], %[p{r}] {rot} row_mask:0xf bank_mask:0xf\\n\\t"',
        f'"v_bfe_u32 %[u], %[s{r}], %[pos], 2\\n\\t"',
        f'"v_cndmask_b32_e64 %[t2], %[{own}], %[{carry}], %[lm]\\n\\t"',
        f'"v_add3_u32 %[c{r}], %[c{r}], %[base], %[u]\\n\\t"',
        f'"v_max3_i32 %[c{r}], %[c{r}], %[p{r}], %[t2]\\n\\t"',
        f'"v_cmp_le_i32 vcc, %[thr], %[c{r}]\\n\\t"',
    ]


def _keep(r):
    """-inf where VCC is clear, then the running maximum."""
    return [
        f'"v_cndmask_b32_e32 %[c{r}], -2.0, %[c{r}], vcc\\n\\t"',
        f'"v_max_i32 %[mx], %[mx], %[c{r}]\\n\\t"',
    ]


def head(C, par, k):
    """Entry block at chain position k: clipped to the entry mask."""
    r = _reg(C, par, k)
    nxt = f".Lr{k + 1}_%=" if k + 1 < C else ".Lend_%="
    return ([f'".Lh{k}_%=:\\n\\t"'] + _cell(C, par, k) + [
        '"s_and_b64 vcc, vcc, %[mf]\\n\\t"',
        '"s_mov_b64 %[lf], vcc\\n\\t"',
    ] + _keep(r) + [
        f'"s_cmp_eq_u32 %[stop], {r}\\n\\t"',
        '"s_cbranch_scc1 .Lend_%=\\n\\t"',
        f'"s_branch {nxt}\\n\\t"',
    ])


def block(C, par, k):
    """Block at chain position k >= 1 of the fall-through run.  The end test
    sits between the compare and its use, as the two wait states the VALU
    needs before reading VCC as a mask."""
    r = _reg(C, par, k)
    return ([f'".Lr{k}_%=:\\n\\t"'] + _cell(C, par, k) + [
        f'"s_cmp_eq_u32 %[stop], {r}\\n\\t"',
        f'"s_cbranch_scc1 .Ll{k}_%=\\n\\t"',
    ] + _keep(r))


def tail(C, par, k):
    """Exit of the block at chain position k when it is the span's last."""
    r = _reg(C, par, k)
    return [f'".Ll{k}_%=:\\n\\t"', '"s_and_b64 vcc, vcc, %[ml]\\n\\t"'] + _keep(r) + [
        '"s_branch .Lend_%=\\n\\t"']


def function(C, par):
    lines = [
        f"template <>",
        f"XD_MEMBER void WChain<{C}, {par}>::run(vint *cur, const vint *prv, const vint *sw,",
        f"                                   int32_t pos, int32_t thr, int32_t base, int32_t rlo,",
        f"                                   int32_t rhi, vint carry, vint &vmx, uint64_t mf,",
        f"                                   uint64_t ml, uint64_t &lf, uint64_t &ll) {{",
        f"  int32_t tA = carry.x, tB = carry.x, t2, u, mx = vmx.x;",
        f"  const int32_t first = {'rlo' if par == 0 else f'{C - 1} - rhi'};   // chain position of the entry",
        f"  const int32_t stop = {'rhi' if par == 0 else 'rlo'};",
        f"  const uint64_t lm = {'1ull' if par == 0 else '1ull << 63'};",
        f"  uint64_t lfv, llv;",
        f"  asm volatile(",
        f'      "s_lshl_b32 s42, %[first], 2\\n\\t"',
        f'      "s_getpc_b64 s[40:41]\\n"',
        f'      ".Lb_%=:\\n\\t"',
        f'      "s_add_u32 s40, s40, s42\\n\\t"',
        f'      "s_addc_u32 s41, s41, 0\\n\\t"',
        f'      "s_add_u32 s40, s40, .Lt_%=-.Lb_%=\\n\\t"',
        f'      "s_addc_u32 s41, s41, 0\\n\\t"',
        f'      "s_nop 0\\n\\t"',
        f'      "s_setpc_b64 s[40:41]\\n"',
        f'      ".Lt_%=:\\n\\t"',
    ]
    for k in range(C):
        lines.append(f'      "s_branch .Lh{k}_%=\\n\\t"')
    for k in range(C):
        lines += ["      " + x for x in head(C, par, k)]
    for k in range(1, C):
        lines += ["      " + x for x in block(C, par, k)]
    lines.append('      "s_branch .Lend_%=\\n\\t"')
    for k in range(1, C):
        lines += ["      " + x for x in tail(C, par, k)]
    lines += ['      ".Lend_%=:\\n\\t"', '      "s_mov_b64 %[ll], vcc\\n"']
    outs = ", ".join(f'[c{r}] "+v"(cur[{r}].x)' for r in range(C))
    ins = ", ".join(f'[p{r}] "v"(prv[{r}].x)' for r in range(C))
    sws = ", ".join(f'[s{r}] "v"(sw[{r}].x)' for r in range(C))
    lines += [
        f"      : {outs},",
        f'        [tA] "+v"(tA), [tB] "+v"(tB), [mx] "+v"(mx), [t2] "=&v"(t2), [u] "=&v"(u),',
        f'        [lf] "=&s"(lfv), [ll] "=&s"(llv)',
        f"      : {ins},",
        f"        {sws},",
        f'        [pos] "s"(pos), [thr] "s"(thr), [base] "s"(base), [first] "s"(first),',
        f'        [stop] "s"(stop), [lm] "s"(lm), [mf] "s"(mf), [ml] "s"(ml)',
        f'      : "vcc", "scc", "s40", "s41", "s42");',
        f"  vmx.x = mx;",
        f"  lf = lfv;",
        f"  ll = llv;",
        f"}}",
        "",
    ]
    return lines


def first_function(C):
    """WFirst<C>::run: slot (64 r + lane) of the first cell above `bw` in
    registers rlo .. rhi, or -1."""
    lines = [
        f"template <>",
        f"XD_MEMBER int32_t WFirst<{C}>::run(const vint *cur, int32_t bw, int32_t rlo, int32_t rhi) {{",
        f"  int32_t slot;",
        f"  asm volatile(",
        f'      "s_lshl_b32 s42, %[rlo], 2\\n\\t"',
        f'      "s_getpc_b64 s[40:41]\\n"',
        f'      ".Lb_%=:\\n\\t"',
        f'      "s_add_u32 s40, s40, s42\\n\\t"',
        f'      "s_addc_u32 s41, s41, 0\\n\\t"',
        f'      "s_add_u32 s40, s40, .Lt_%=-.Lb_%=\\n\\t"',
        f'      "s_addc_u32 s41, s41, 0\\n\\t"',
        f'      "s_nop 0\\n\\t"',
        f'      "s_setpc_b64 s[40:41]\\n"',
        f'      ".Lt_%=:\\n\\t"',
    ]
    for r in range(C):
        lines.append(f'      "s_branch .Lq{r}_%=\\n\\t"')
    for r in range(C):
        lines += [
            f'      ".Lq{r}_%=:\\n\\t"',
            f'      "v_cmp_lt_i32_e32 vcc, %[bw], %[c{r}]\\n\\t"',
            f'      "s_cbranch_vccnz .Lf{r}_%=\\n\\t"',
            f'      "s_cmp_eq_u32 %[rhi], {r}\\n\\t"',
            f'      "s_cbranch_scc1 .Lnone_%=\\n\\t"',
        ]
    lines += [
        '      ".Lnone_%=:\\n\\t"',
        '      "s_mov_b32 %[slot], -1\\n\\t"',
        '      "s_branch .Lend_%=\\n\\t"',
    ]
    for r in range(C):
        lines += [
            f'      ".Lf{r}_%=:\\n\\t"',
            '      "s_ff1_i32_b64 %[slot], vcc\\n\\t"',
            f'      "s_add_i32 %[slot], %[slot], {64 * r}\\n\\t"',
            '      "s_branch .Lend_%=\\n\\t"',
        ]
    ins = ", ".join(f'[c{r}] "v"(cur[{r}].x)' for r in range(C))
    lines += [
        '      ".Lend_%=:\\n"',
        '      : [slot] "=&s"(slot)',
        f"      : {ins},",
        '        [bw] "s"(bw), [rlo] "s"(rlo), [rhi] "s"(rhi)',
        '      : "vcc", "scc", "s40", "s41", "s42");',
        "  return slot;",
        "}",
        "",
    ]
    return lines


def render() -> str:
    """The header's text."""
    out = [
        "// xd_wchain_asm.h -- generated by gen_wchain.py; do not edit.",
        "//",
        "// The register chain of the wide tiers (wcell_chain in xd_wide.h) as",
        "// gfx950 assembly for narrow score fields: WChain<C, PAR>::run updates",
        "// registers rlo..rhi of the span (upwards on even anti-diagonals,",
        "// downwards on odd ones), clips the entry register to the lanes in mf",
        "// and the last one to those in ml (cells outside become -inf), and folds",
        "// each register into the running maximum vmx.  lf and ll return the",
        "// survivors of the entry and the last register (the same register when",
        "// rlo == rhi; mf then holds both clips).  `carry` is the outer neighbour",
        "// rotation of the chain's first register.  Reads only registers; writes",
        "// only cur[rlo..rhi].",
        "//",
        "// WFirst<C>::run returns the first slot (64 r + lane) of registers",
        "// rlo..rhi whose cell exceeds bw, or -1 when none does.",
        "#pragma once",
        "",
        '#include "xd_wave.h"',
        "",
        "namespace xd {",
        "",
        "template <int C, int PAR>",
        "struct WChain {",
        "  XD_MEMBER static void run(vint *cur, const vint *prv, const vint *sw, int32_t pos,",
        "                            int32_t thr, int32_t base, int32_t rlo, int32_t rhi,",
        "                            vint carry, vint &vmx, uint64_t mf, uint64_t ml,",
        "                            uint64_t &lf, uint64_t &ll);",
        "};",
        "",
        "template <int C>",
        "struct WFirst {",
        "  XD_MEMBER static int32_t run(const vint *cur, int32_t bw, int32_t rlo, int32_t rhi);",
        "};",
        "",
    ]
    for C in CS:
        for par in (0, 1):
            out += function(C, par)
        out += first_function(C)
    out += ["}  // namespace xd", ""]
    return "\n".join(out)


def main():
    with open(os.path.join(HERE, "xd_wchain_asm.h"), "w") as f:
        f.write(render())


if __name__ == "__main__":
    main()
