"""The generated register-chain assembly (csrc/xd_wchain_asm.h) is what its
generator writes, and every block of it has the shape the wide tiers rely on."""
import importlib.util
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2002_05200_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_wchain", os.path.join(CSRC, "gen_wchain.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_header_matches_generator():
    with open(os.path.join(CSRC, "xd_wchain_asm.h")) as f:
        assert f.read() == _gen().render(), "regenerate: python paper_2002_05200_amd/csrc/gen_wchain.py"


def test_every_register_count_and_parity_is_generated():
    text = _gen().render()
    for c in (2, 4, 8, 16, 32):
        for par in (0, 1):
            assert f"WChain<{c}, {par}>::run" in text


def _blocks(lines):
    """Label -> the instructions under it, in order of appearance."""
    out, cur = [], None
    for ln in lines.split("\n"):
        m = re.search(r'"\.L([hrl])(\d+)_%=:', ln)
        if m:
            cur = (m.group(1), int(m.group(2)), [])
            out.append(cur)
        elif '".Lend_%=:' in ln:
            cur = None
        elif cur is not None:
            cur[2].append(ln)
    return out


def test_chain_order_end_tests_and_clipping():
    gen = _gen()
    for c in (4, 32):
        for par in (0, 1):
            text = "\n".join(gen.function(c, par))
            reg = (lambda k: k) if par == 0 else (lambda k: c - 1 - k)
            blocks = _blocks(text)
            kinds = [(kind, k) for kind, k, _ in blocks]
            # a head per entry position, then the fall-through run from
            # position 1, then a tail per position that can end the chain
            assert kinds == ([("h", k) for k in range(c)] + [("r", k) for k in range(1, c)]
                             + [("l", k) for k in range(1, c)])
            for kind, k, body in blocks:
                code = "\n".join(body)
                r = reg(k)
                if kind in "hr":
                    assert re.findall(r"v_max3_i32 %\[c(\d+)\]", code) == [str(r)]
                    # the block ends the chain when it reaches the span's other end
                    assert re.findall(r"s_cmp_eq_u32 %\[stop\], (\d+)", code) == [str(r)]
                    # neighbour rotation: right for even anti-diagonals, left for odd
                    assert code.count("wave_ror:1" if par == 0 else "wave_rol:1") == 1
                    # the X-drop test comes two instructions before its use as a mask
                    ins = [b.strip().strip('"').split()[0] for b in body]
                    i_cmp = ins.index("v_cmp_le_i32")
                    i_use = ins.index("v_cndmask_b32_e32")
                    assert i_use - i_cmp >= 3
                if kind == "h":
                    # the entry register is clipped to mf and its survivors kept
                    assert "s_and_b64 vcc, vcc, %[mf]" in code and "s_mov_b64 %[lf], vcc" in code
                    assert code.index("%[mf]") < code.index("v_cndmask_b32_e32")
                    nxt = f".Lr{k + 1}_%=" if k + 1 < c else ".Lend_%="
                    assert body[-1].strip().startswith(f'"s_branch {nxt}')
                if kind == "r":
                    assert f"s_cbranch_scc1 .Ll{k}_%=" in code and "%[mf]" not in code
                    assert "%[ml]" not in code
                if kind == "l":
                    # the last register is clipped to ml before -inf and the maximum
                    assert code.index("s_and_b64 vcc, vcc, %[ml]") < code.index("v_cndmask")
                    assert f"%[c{r}]" in code
            # the last register's survivors are what VCC holds at the end
            assert text.rstrip().count('"s_mov_b64 %[ll], vcc') == 1


def test_first_best_scan_shape():
    """WFirst<C>: entered at rlo through a table, each register is one
    compare of bw < cell and a branch to its own found-stub, then the end
    test against rhi; a found-stub returns the lowest set lane + 64 r."""
    gen = _gen()
    for c in (4, 16):
        text = "\n".join(gen.first_function(c))
        table = re.findall(r'"s_branch \.Lq(\d+)_%=', text)
        assert [int(x) for x in table] == list(range(c))
        scans = re.findall(r"v_cmp_lt_i32_e32 vcc, %\[bw\], %\[c(\d+)\]", text)
        assert [int(x) for x in scans] == list(range(c))
        assert [int(x) for x in re.findall(r"s_cbranch_vccnz \.Lf(\d+)_%=", text)] == list(range(c))
        assert [int(x) for x in re.findall(r"s_cmp_eq_u32 %\[rhi\], (\d+)", text)] == list(range(c))
        offs = [int(x) for x in re.findall(r"s_add_i32 %\[slot\], %\[slot\], (\d+)", text)]
        assert offs == [64 * r for r in range(c)]
        assert text.count("s_ff1_i32_b64 %[slot], vcc") == c
        # no register found: -1
        assert '"s_mov_b32 %[slot], -1' in text
