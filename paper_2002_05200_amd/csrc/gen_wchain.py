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
import re

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


def function_run(C, par):
    """WChainRun<C, PAR>::run: WChain's chain run to the window's last
    register (C - 1 going up, 0 going down) without a test per register; the
    far register of the range (rhi going up, rlo going down) is then cut to
    the lanes in ml through a table of branches, its survivors go to ll, and
    the register past it becomes -inf.  Past the span's far end every input
    is -inf except for at most two slots next to it when the range was
    clipped there, so the registers beyond need nothing more; lanes cut from
    the far register may have raised vmx, which callers only use to start a
    search of the range itself."""
    stop = "rhi" if par == 0 else "rlo"
    lines = [
        f"template <>",
        f"XD_MEMBER void WChainRun<{C}, {par}>::run(vint *cur, const vint *prv, const vint *sw,",
        f"                                      int32_t pos, int32_t thr, int32_t base, int32_t rlo,",
        f"                                      int32_t rhi, vint carry, vint &vmx, uint64_t mf,",
        f"                                      uint64_t ml, uint64_t &lf, uint64_t &ll) {{",
        f"  int32_t tA = carry.x, tB = carry.x, t2, u, mx = vmx.x;",
        f"  const int32_t first = {'rlo' if par == 0 else f'{C - 1} - rhi'};   // chain position of the entry",
        f"  const int32_t stop = {stop};",
        f"  const uint64_t lm = {'1ull' if par == 0 else '1ull << 63'};",
        f"  uint64_t lfv, llv;",
        f"  asm volatile(",
    ]
    body = [x.replace("{t}", ".Lj") for x in _jump(".Lh{}_%=", "first", C)]
    for k in range(C):
        r = _reg(C, par, k)
        nxt = f".Lr{k + 1}_%=" if k + 1 < C else ".Lfx_%="
        body += [f'".Lh{k}_%=:\\n\\t"'] + _cell(C, par, k) + [
            '"s_and_b64 vcc, vcc, %[mf]\\n\\t"',
            '"s_mov_b64 %[lf], vcc\\n\\t"',
        ] + _keep(r) + [f'"s_branch {nxt}\\n\\t"']
    for k in range(1, C):
        body += [f'".Lr{k}_%=:\\n\\t"'] + _cell(C, par, k) + _keep(_reg(C, par, k))
    body += ['".Lfx_%=:\\n\\t"']
    body += [x.replace("{t}", ".Lx") for x in _jump(".LF{}_%=", "stop", C)]
    for r in range(C):
        rn = r + 1 if par == 0 else r - 1
        body += [
            f'".LF{r}_%=:\\n\\t"',
            f'"v_cndmask_b32_e64 %[c{r}], -2.0, %[c{r}], %[ml]\\n\\t"',
            f'"v_cmp_le_i32_e64 %[ll], %[thr], %[c{r}]\\n\\t"',
        ] + ([f'"v_mov_b32 %[c{rn}], -2.0\\n\\t"'] if 0 <= rn < C else []) + [
            '"s_branch .Lend_%=\\n\\t"',
        ]
    body += ['".Lend_%=:\\n"']
    lines += ["      " + x for x in body]
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


# ---------------------------------------------------------------------------
# WLoop<C>::run: whole anti-diagonals of one score-word block in assembly
# ---------------------------------------------------------------------------
def _jump(label_fmt, idx, n):
    """A table of n branches indexed by SGPR operand `idx` (entry k jumps to
    label_fmt.format(k))."""
    out = [
        f'"s_lshl_b32 s42, %[{idx}], 2\\n\\t"',
        '"s_getpc_b64 s[40:41]\\n"',
        '"{t}b_%=:\\n\\t"',
        '"s_add_u32 s40, s40, s42\\n\\t"',
        '"s_addc_u32 s41, s41, 0\\n\\t"',
        '"s_add_u32 s40, s40, {t}t_%=-{t}b_%=\\n\\t"',
        '"s_addc_u32 s41, s41, 0\\n\\t"',
        '"s_nop 0\\n\\t"',
        '"s_setpc_b64 s[40:41]\\n"',
        '"{t}t_%=:\\n\\t"',
    ]
    out += [f'"s_branch {label_fmt.format(k)}\\n\\t"' for k in range(n)]
    return out


def _loop_chain(C, par, P):
    """The chain of one parity inside WLoop (labels prefixed with P): cur
    registers are c{r} (even: E, odd: O), the previous anti-diagonal's are
    p{r}, score words w{r}.

    Both parities walk the span downwards, from rhi to the window's register
    0, without a test per register.  A cell's neighbour on the previous
    anti-diagonal is the rotation of its own register with one lane taken
    from the register beside it: on even anti-diagonals slot s - 1 (lane 0
    from the register below, whose rotation each block computes for itself
    and leaves to the next block as that block's own rotation), on odd ones
    slot s + 1 (lane 63 from the register above, rotated by the block
    before).  The entry register takes that neighbour from the real register
    (a live cell when the range was clipped to the matrix there), is cut to
    the range (mask mf) before the X-drop test, and its survivors go
    straight to lf.  Below the span's low end every input is -inf except for
    at most two slots next to it (cells a clipped range left out of the
    matrix), so the registers there stay -inf but for those slots; the low
    edge register rlo and the one below it are put right afterwards through
    a table of branches on rlo: the edge register is cut to the range (mask
    ml) and its survivors go to ll, the register below it becomes -inf (it
    lies outside the span).  Cut lanes may have raised the running maximum:
    the improvement search that follows only looks at the range, so such a
    false alarm changes nothing.  Placing bands low in the window keeps the
    registers below the span few."""
    cur = "e" if par == 0 else "o"
    prv = "o" if par == 0 else "e"
    sw = "se" if par == 0 else "so"
    rot = "wave_ror:1" if par == 0 else "wave_rol:1"

    def reg(k):
        return C - 1 - k

    def regs(k):
        """(rotation written by block k, the other one) for position k."""
        return ("tA", "tB") if k % 2 == 0 else ("tB", "tA")

    def cell(k, cond="vcc", mask=None):
        r = reg(k)
        mine, other = regs(k)
        cmp = (f'"v_cmp_le_i32 vcc, %[thr], %[{cur}{r}]\\n\\t"' if cond == "vcc" else
               f'"v_cmp_le_i32_e64 %[{cond}], %[thr], %[{cur}{r}]\\n\\t"')
        cut = ([f'"v_cndmask_b32_e64 %[{cur}{r}], -2.0, %[{cur}{r}], %[{mask}]\\n\\t"']
               if mask else [])
        if par == 0:
            # even: this block rotates the register below (lane 0's neighbour here,
            # the next block's own rotation); its own rotation is in `other`
            below = (f'"v_mov_b32_dpp %[{mine}], %[{prv}{r - 1}] {rot} row_mask:0xf bank_mask:0xf\\n\\t"'
                     if r >= 1 else f'"v_mov_b32 %[{mine}], -2.0\\n\\t"')
            nbr = [below, f'"v_bfe_u32 %[u], %[{sw}{r}], %[pos], 2\\n\\t"',
                   f'"v_cndmask_b32_e64 %[t2], %[{other}], %[{mine}], %[lm0]\\n\\t"']
        else:
            # odd: this block rotates its own register; lane 63's neighbour is the
            # rotation of the register above, left by the block before in `other`
            nbr = [f'"v_mov_b32_dpp %[{mine}], %[{prv}{r}] {rot} row_mask:0xf bank_mask:0xf\\n\\t"',
                   f'"v_bfe_u32 %[u], %[{sw}{r}], %[pos], 2\\n\\t"',
                   f'"v_cndmask_b32_e64 %[t2], %[{mine}], %[{other}], %[lm1]\\n\\t"']
        return nbr + [
            f'"v_add3_u32 %[{cur}{r}], %[{cur}{r}], %[base], %[u]\\n\\t"',
            f'"v_max3_i32 %[{cur}{r}], %[{cur}{r}], %[{prv}{r}], %[t2]\\n\\t"',
        ] + cut + [cmp]

    def keep(k, cond="vcc"):
        r = reg(k)
        sel = (f'"v_cndmask_b32_e32 %[{cur}{r}], -2.0, %[{cur}{r}], vcc\\n\\t"' if cond == "vcc" else
               f'"v_cndmask_b32_e64 %[{cur}{r}], -2.0, %[{cur}{r}], %[{cond}]\\n\\t"')
        return [sel, f'"v_max_i32 %[mx], %[mx], %[{cur}{r}]\\n\\t"']

    out = [
        '"v_mov_b32 %[tA], -2.0\\n\\t"',     # the neighbour above the window: -inf
        '"v_mov_b32 %[tB], -2.0\\n\\t"',
        '"v_mov_b32 %[mx], -2.0\\n\\t"',
        f'"s_sub_u32 %[ix], {C - 1}, %[rhi]\\n\\t"',   # chain position of rhi
    ]
    out += [x.replace("{t}", f".L{P}j") for x in _jump(f".L{P}h{{}}_%=", "ix", C)]
    for k in range(C):
        r = reg(k)
        mine, other = regs(k)
        nxt = f".L{P}r{k + 1}_%=" if k + 1 < C else f".L{P}fx_%="
        out += [f'".L{P}h{k}_%=:\\n\\t"']
        if par == 0:   # the entry's own rotation (the block before would have left it)
            out += [f'"v_mov_b32_dpp %[{other}], %[{prv}{r}] {rot} row_mask:0xf bank_mask:0xf\\n\\t"']
        elif r + 1 < C:   # the rotation of the register above the entry
            out += [f'"v_mov_b32_dpp %[{other}], %[{prv}{r + 1}] {rot} row_mask:0xf bank_mask:0xf\\n\\t"']
        out += cell(k, "lf", "mf") + keep(k, "lf") + [f'"s_branch {nxt}\\n\\t"']
    for k in range(1, C):
        out += [f'".L{P}r{k}_%=:\\n\\t"'] + cell(k) + keep(k)
    # the low edge register rlo and the one below it
    out += [f'".L{P}fx_%=:\\n\\t"']
    out += [x.replace("{t}", f".L{P}x") for x in _jump(f".L{P}F{{}}_%=", "rlo", C)]
    for r in range(C):
        out += [
            f'".L{P}F{r}_%=:\\n\\t"',
            f'"v_cndmask_b32_e64 %[{cur}{r}], -2.0, %[{cur}{r}], %[ml]\\n\\t"',
            f'"v_cmp_le_i32_e64 %[ll], %[thr], %[{cur}{r}]\\n\\t"',
        ] + ([f'"v_mov_b32 %[{cur}{r - 1}], -2.0\\n\\t"'] if r >= 1 else []) + [
            f'"s_branch .L{P}end_%=\\n\\t"',
        ]
    out += [f'".L{P}end_%=:\\n\\t"']
    return out


def _loop_half(C, par):
    """One anti-diagonal of parity `par` in WLoop, from the block-end test to
    the recentre test of the next range."""
    P = "E" if par == 0 else "O"
    cur = "e" if par == 0 else "o"
    spl, sph = f"spl{par}", f"sph{par}"
    out = [f'".L{P}top_%=:\\n\\t"']
    if par == 0:   # a block ends before an even anti-diagonal
        out += ['"s_cmp_ge_i32 %[d], %[dstop]\\n\\t"', '"s_cbranch_scc1 .Lx0_%=\\n\\t"']
    out += [
        '"s_ashr_i32 %[rlo], %[lo], 6\\n\\t"',
        '"s_ashr_i32 %[rhi], %[hi], 6\\n\\t"',
        # registers leaving this parity's span become -inf (out of line)
        f'"s_cmp_lt_i32 %[{spl}], %[rlo]\\n\\t"',
        f'"s_cbranch_scc1 .L{P}cl_%=\\n\\t"',
        f'"s_cmp_gt_i32 %[{sph}], %[rhi]\\n\\t"',
        f'"s_cbranch_scc1 .L{P}cl_%=\\n"',
        f'".L{P}clret_%=:\\n\\t"',
        # lane masks of the range in its edge registers
        '"s_and_b32 %[t], %[lo], 63\\n\\t"',
        '"s_lshl_b64 %[mlo], -1, %[t]\\n\\t"',
        '"s_and_b32 %[t], %[hi], 63\\n\\t"',
        '"s_sub_u32 %[t], 63, %[t]\\n\\t"',
        '"s_lshr_b64 %[mhi], -1, %[t]\\n\\t"',
        '"s_and_b64 %[mf], %[mlo], %[mhi]\\n\\t"',
        '"s_cmp_eq_u32 %[rlo], %[rhi]\\n\\t"',
    ]
    # the chain enters at rhi (mask hi) and leaves at rlo (mask lo)
    out += ['"s_cselect_b64 %[mf], %[mf], %[mhi]\\n\\t"', '"s_mov_b64 %[ml], %[mlo]\\n\\t"',
            '"s_sub_i32 %[pos], %[d], %[e0x2]\\n\\t"']
    if par == 1:
        out += ['"s_add_i32 %[pos], %[pos], -1\\n\\t"']
    out += _loop_chain(C, par, P)
    # survivors of the range's first and last register
    # (lf, the entry register's, was written long before ll: test it first)
    lo_mask, hi_mask = "ll", "lf"
    first_part = [
        f'"s_cmp_eq_u64 %[{lo_mask}], 0\\n\\t"',
        '"s_cbranch_scc1 .Lx2_%=\\n\\t"',
        f'"s_ff1_i32_b64 %[first], %[{lo_mask}]\\n\\t"',
        '"s_lshl_b32 %[t], %[rlo], 6\\n\\t"',
        '"s_add_i32 %[first], %[first], %[t]\\n\\t"',
    ]
    last_part = [
        f'"s_cmp_eq_u64 %[{hi_mask}], 0\\n\\t"',
        '"s_cbranch_scc1 .Lx2_%=\\n\\t"',
        f'"s_flbit_i32_b64 %[last], %[{hi_mask}]\\n\\t"',
        '"s_lshl_b32 %[t], %[rhi], 6\\n\\t"',
        '"s_add_i32 %[t], %[t], 63\\n\\t"',
        '"s_sub_i32 %[last], %[t], %[last]\\n\\t"',
    ]
    out += last_part + first_part
    out += [
        # did best improve?  (match = 1: by exactly one; out of line)
        '"v_cmp_lt_i32_e32 vcc, %[bw], %[mx]\\n\\t"',
        f'"s_cbranch_vccnz .L{P}imp_%=\\n"',
        f'".L{P}impret_%=:\\n\\t"',
        # cells of this range, the span of this parity
        '"s_sub_i32 %[t], %[hi], %[lo]\\n\\t"',
        '"s_add_i32 %[cells], %[cells], %[t]\\n\\t"',
        '"s_add_i32 %[cells], %[cells], 1\\n\\t"',
        f'"s_mov_b32 %[{spl}], %[rlo]\\n\\t"',
        f'"s_mov_b32 %[{sph}], %[rhi]\\n\\t"',
    ]
    if par == 0:   # next (odd) range: [first - 1, last]
        out += ['"s_add_i32 %[lo], %[first], -1\\n\\t"', '"s_mov_b32 %[hi], %[last]\\n\\t"']
    else:          # next (even) range: [first, last + 1]
        out += ['"s_mov_b32 %[lo], %[first]\\n\\t"', '"s_add_i32 %[hi], %[last], 1\\n\\t"']
    out += [
        '"s_add_i32 %[bw], %[bw], %[ng]\\n\\t"',
        '"s_add_i32 %[thr], %[thr], %[ng]\\n\\t"',
        '"s_add_i32 %[d], %[d], 1\\n\\t"',
        # clipped to the matrix: j <= n (slot >= floor(d/2) - n - h) and
        # i <= m (slot <= m - h - ceil(d/2)); empty: the extension ends
        '"s_lshr_b32 %[t], %[d], 1\\n\\t"',
        '"s_sub_i32 %[t], %[t], %[nh]\\n\\t"',
        '"s_max_i32 %[lo], %[lo], %[t]\\n\\t"',
        '"s_add_i32 %[t], %[d], 1\\n\\t"',
        '"s_lshr_b32 %[t], %[t], 1\\n\\t"',
        '"s_sub_i32 %[t], %[mh], %[t]\\n\\t"',
        '"s_min_i32 %[hi], %[hi], %[t]\\n\\t"',
        '"s_cmp_gt_i32 %[lo], %[hi]\\n\\t"',
        '"s_cbranch_scc1 .Lx4_%=\\n\\t"',
        '"s_cmp_lt_i32 %[lo], 1\\n\\t"',
        '"s_cbranch_scc1 .Lx3_%=\\n\\t"',
        '"s_cmp_gt_i32 %[hi], %[smax]\\n\\t"',
        '"s_cbranch_scc1 .Lx3_%=\\n\\t"',
    ]
    return out


def _loop_outofline(C, par):
    """Span clearing and the improvement search of one parity."""
    P = "E" if par == 0 else "O"
    cur = "e" if par == 0 else "o"
    spl, sph = f"spl{par}", f"sph{par}"
    out = [
        # clear registers of the old span [spl, sph] that are outside [rlo, rhi]
        f'".L{P}cl_%=:\\n\\t"',
        f'"s_mov_b32 %[ix], %[{spl}]\\n"',
        f'".L{P}clloop_%=:\\n\\t"',
        f'"s_cmp_gt_i32 %[ix], %[{sph}]\\n\\t"',
        f'"s_cbranch_scc1 .L{P}clret_%=\\n\\t"',
        '"s_cmp_lt_i32 %[ix], %[rlo]\\n\\t"',
        f'"s_cbranch_scc1 .L{P}cldo_%=\\n\\t"',
        '"s_cmp_gt_i32 %[ix], %[rhi]\\n\\t"',
        f'"s_cbranch_scc1 .L{P}cldo_%=\\n"',
        f'".L{P}clnext_%=:\\n\\t"',
        '"s_add_i32 %[ix], %[ix], 1\\n\\t"',
        f'"s_branch .L{P}clloop_%=\\n"',
        f'".L{P}cldo_%=:\\n\\t"',
    ]
    out += [x.replace("{t}", f".L{P}z") for x in _jump(f".L{P}z{{}}_%=", "ix", C)]
    for r in range(C):
        out += [f'".L{P}z{r}_%=:\\n\\t"', f'"v_mov_b32 %[{cur}{r}], -2.0\\n\\t"',
                f'"s_branch .L{P}clnext_%=\\n\\t"']
    # improvement: the first slot above bw, scanning the span upwards
    out += [f'".L{P}imp_%=:\\n\\t"']
    out += [x.replace("{t}", f".L{P}q") for x in _jump(f".L{P}q{{}}_%=", "rlo", C)]
    for r in range(C):
        out += [
            f'".L{P}q{r}_%=:\\n\\t"',
            f'"v_cmp_lt_i32_e32 vcc, %[bw], %[{cur}{r}]\\n\\t"',
            f'"s_cbranch_vccnz .L{P}f{r}_%=\\n\\t"',
            f'"s_cmp_eq_u32 %[rhi], {r}\\n\\t"',
            f'"s_cbranch_scc1 .L{P}impret_%=\\n\\t"',
        ]
    out.append(f'"s_branch .L{P}impret_%=\\n\\t"')
    for r in range(C):
        out += [
            f'".L{P}f{r}_%=:\\n\\t"',
            '"s_ff1_i32_b64 %[bs], vcc\\n\\t"',
            f'"s_add_i32 %[bs], %[bs], {64 * r}\\n\\t"',
            '"s_mov_b32 %[bpos], %[d]\\n\\t"',
            '"s_add_i32 %[bw], %[bw], 1\\n\\t"',
            '"s_add_i32 %[thr], %[thr], 1\\n\\t"',
            f'"s_branch .L{P}impret_%=\\n\\t"',
        ]
    return out


def loop_function(C, fold=False):
    """WLoop<C, FOLD>::run: anti-diagonals of the current score-word block
    (score words built for every register), with match = 1 and narrow score
    fields, each range clipped to the matrix.  Returns why it stopped: 0 the
    block ended, 2 anti-diagonal s.d has been computed but its survivors are
    not in the span's edge registers (the caller finishes it), 3 the next
    range needs a recentre, 4 the next range lies outside the matrix (the
    extension has ended).  FOLD: the score fields hold base + delta * match
    themselves (+1/-1/-1), so the diagonal term is one VOP2 add."""
    lines = [
        "template <>",
        f"XD_MEMBER int32_t WLoop<{C}, {'true' if fold else 'false'}>::run(vint *E, vint *O, const vint *SE, const vint *SO,",
        "                                   WLoopState &s) {",
        "  int32_t d = s.d, lo = s.lo, hi = s.hi, bw = s.bw, thr = s.thr, cells = s.cells;",
        "  int32_t bs = s.bs, bpos = s.bpos, spl0 = s.spl0, sph0 = s.sph0, spl1 = s.spl1, sph1 = s.sph1;",
        "  int32_t rlo = 0, rhi = 0, code = 0, ix, t, pos, first, last;",
        "  uint64_t mlo, mhi, mf, ml, lf = 0, ll = 0;",
        "  const uint64_t lm0 = 1ull, lm1 = 1ull << 63;",
        "  int32_t tA, tB, t2, u, mx = -(1 << 30);",
        "  asm volatile(",
        '      "s_bitcmp1_b32 %[d], 0\\n\\t"',
        '      "s_cbranch_scc1 .LOtop_%=\\n\\t"',
    ]
    body = _loop_half(C, 0) + _loop_half(C, 1) + ['"s_branch .LEtop_%=\\n"']
    body += [
        '".Lx0_%=:\\n\\t"', '"s_mov_b32 %[code], 0\\n\\t"', '"s_branch .Lend_%=\\n"',
        '".Lx2_%=:\\n\\t"', '"s_mov_b32 %[code], 2\\n\\t"', '"s_branch .Lend_%=\\n"',
        '".Lx3_%=:\\n\\t"', '"s_mov_b32 %[code], 3\\n\\t"', '"s_branch .Lend_%=\\n"',
        '".Lx4_%=:\\n\\t"', '"s_mov_b32 %[code], 4\\n\\t"', '"s_branch .Lend_%=\\n"',
    ]
    body += _loop_outofline(C, 0) + _loop_outofline(C, 1)
    body += ['".Lend_%=:\\n"']
    if fold:
        body = [re.sub(r"v_add3_u32 %\[(\w+)\], %\[\1\], %\[base\], %\[u\]",
                       r"v_add_u32 %[\1], %[u], %[\1]", x) for x in body]
    lines += ["      " + x for x in body]
    outs = ", ".join([f'[e{r}] "+v"(E[{r}].x)' for r in range(C)] +
                     [f'[o{r}] "+v"(O[{r}].x)' for r in range(C)])
    ins = ", ".join([f'[se{r}] "v"(SE[{r}].x)' for r in range(C)] +
                    [f'[so{r}] "v"(SO[{r}].x)' for r in range(C)])
    lines += [
        f"      : {outs},",
        '        [tA] "=&v"(tA), [tB] "=&v"(tB), [t2] "=&v"(t2), [u] "=&v"(u), [mx] "+v"(mx),',
        '        [d] "+s"(d), [lo] "+s"(lo), [hi] "+s"(hi), [bw] "+s"(bw), [thr] "+s"(thr),',
        '        [cells] "+s"(cells), [bs] "+s"(bs), [bpos] "+s"(bpos), [spl0] "+s"(spl0),',
        '        [sph0] "+s"(sph0), [spl1] "+s"(spl1), [sph1] "+s"(sph1), [rlo] "+s"(rlo),',
        '        [rhi] "+s"(rhi), [code] "+s"(code), [ix] "=&s"(ix), [t] "=&s"(t),',
        '        [pos] "=&s"(pos), [first] "=&s"(first), [last] "=&s"(last), [mlo] "=&s"(mlo),',
        '        [mhi] "=&s"(mhi), [mf] "=&s"(mf), [ml] "=&s"(ml), [lf] "+s"(lf), [ll] "+s"(ll)',
        f"      : {ins},",
        '        [dstop] "s"(s.dstop), [e0x2] "s"(s.e0x2), [mh] "s"(s.mh), [nh] "s"(s.nh),',
        '        [base] "s"(s.base), [ng] "s"(s.ng), [smax] "s"(s.smax), [lm0] "s"(lm0),',
        '        [lm1] "s"(lm1)',
        '      : "vcc", "scc", "s40", "s41", "s42");',
        "  s.d = d; s.lo = lo; s.hi = hi; s.bw = bw; s.thr = thr; s.cells = cells;",
        "  s.bs = bs; s.bpos = bpos; s.spl0 = spl0; s.sph0 = sph0; s.spl1 = spl1; s.sph1 = sph1;",
        "  s.rlo = rlo; s.rhi = rhi; s.lf = lf; s.ll = ll; s.mx = mx;",
        "  return code;",
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
        "//",
        "// WChainRun<C, PAR>::run is the same chain run to the window's last",
        "// register without a test per register, the far register cut to ml",
        "// afterwards and the register past it set to -inf; its vmx may count",
        "// lanes past the range (callers search the range itself).",
        "//",
        "// WLoop<C, FOLD>::run runs whole anti-diagonals of one score-word block",
        "// (FOLD: the fields hold base + delta * match, +1/-1/-1):",
        "// span clearing, the chain, survivors, the improvement of best (match =",
        "// 1), cells and the next range clipped to the matrix, leaving when the",
        "// block ends, the survivors are not in the span's edge registers, the",
        "// next range needs a recentre, or the clipped range is empty.",
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
        "template <int C, int PAR>",
        "struct WChainRun {",
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
        "// Scalar state of WLoop: the anti-diagonal about to be computed, its range",
        "// (slots), the W-form thresholds, cells of the block, the last improvement",
        "// (slot and anti-diagonal, bpos = -1 for none) and both parities' spans;",
        "// the block's limits; and, after a return of 2, the finished chain's span,",
        "// edge survivors and running maximum.",
        "struct WLoopState {",
        "  int32_t d, lo, hi, bw, thr, cells, bs, bpos, spl0, sph0, spl1, sph1;",
        "  int32_t dstop, e0x2, mh, nh, base, ng, smax;   // mh = m - h, nh = n + h",
        "  int32_t rlo, rhi;",
        "  uint64_t lf, ll;",
        "  int32_t mx;",
        "};",
        "",
        "template <int C, bool FOLD>",
        "struct WLoop {",
        "  XD_MEMBER static int32_t run(vint *E, vint *O, const vint *SE, const vint *SO,",
        "                              WLoopState &s);",
        "};",
        "",
    ]
    for C in CS:
        for par in (0, 1):
            out += function(C, par)
            out += function_run(C, par)
        out += first_function(C)
        if C >= 4:
            out += loop_function(C)
            out += loop_function(C, True)
    out += ["}  // namespace xd", ""]
    return "\n".join(out)


def main():
    with open(os.path.join(HERE, "xd_wchain_asm.h"), "w") as f:
        f.write(render())


if __name__ == "__main__":
    main()
