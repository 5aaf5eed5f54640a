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


def test_chain_order_and_end_tests():
    gen = _gen()
    for c in (4, 32):
        for par in (0, 1):
            lines = "\n".join(gen.function(c, par))
            regs = [int(r) for r in re.findall(r"v_max3_i32 %\[c(\d+)\]", lines)]
            assert regs == (list(range(c)) if par == 0 else list(range(c - 1, -1, -1)))
            # each block ends the chain when it reaches the span's other end
            stops = [int(r) for r in re.findall(r"s_cmp_eq_u32 %\[stop\], (\d+)", lines)]
            assert stops == regs
            # neighbour rotation: right for even anti-diagonals, left for odd
            assert lines.count("wave_ror:1" if par == 0 else "wave_rol:1") == c
