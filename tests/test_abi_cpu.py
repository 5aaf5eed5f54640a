"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function the header declares, and its host-only entry points behave."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xdrop.h")


@pytest.fixture(scope="module")
def L():
    from paper_2002_05200_amd import build
    if not os.path.exists(build.LIB):
        build.build(verbose=False)
    from paper_2002_05200_amd import xdrop
    return xdrop.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(xd[a-z_]*)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["xdrop_extend", "xdrop_extend_host", "xd_pack", "xd_pack_codes", "xd_ctx_create",
              "xd_ctx_destroy", "xd_last_error", "xd_last_stats", "xd_server_create",
              "xd_server_submit", "xd_server_poll", "xd_server_get_stats", "xd_server_destroy"]:
        assert n in names


def test_every_declared_symbol_is_exported(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_single_hip_runtime_in_process(L):
    maps = open("/proc/self/maps").read()
    libs = {l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l}
    assert len(libs) == 1, libs


def test_pack_ascii_matches_layout():
    from paper_2002_05200_amd import synth, xdrop
    r = np.random.default_rng(3)
    for n in [0, 1, 15, 16, 17, 100, 1000]:
        codes = r.integers(0, 4, n).astype(np.uint8)
        text = synth.decode(codes)
        w = xdrop.pack_ascii(text)
        w2 = xdrop.pack_codes(codes)
        assert np.array_equal(w, w2)
        # base g in bits [2(g%16), 2(g%16)+1] of word g/16
        for g in range(n):
            assert (int(w[g // 16]) >> (2 * (g % 16))) & 3 == codes[g]
        assert xdrop.pack_ascii(text.lower()).tolist() == w.tolist()


def test_pack_rejects_non_acgt():
    from paper_2002_05200_amd import xdrop
    with pytest.raises(xdrop.XdropError) as e:
        xdrop.pack_ascii(b"ACGTN")
    assert e.value.status == xdrop.XD_EINVAL
    assert "not ACGT" in xdrop.last_error()
    with pytest.raises(xdrop.XdropError):
        xdrop.pack_codes(np.array([0, 1, 4], np.uint8))


def test_pack_codes_at_offset_preserves_neighbours(L):
    words = np.full(4, 0xFFFFFFFF, dtype=np.uint32)
    codes = np.array([0, 1, 2, 3, 0], np.uint8)
    rc = L.xd_pack_codes(codes.ctypes.data_as(ctypes.c_void_p), len(codes),
                         words.ctypes.data_as(ctypes.c_void_p), 14)
    assert rc == 0
    got = [(int(words[(14 + t) // 16]) >> (2 * ((14 + t) % 16))) & 3 for t in range(5)]
    assert got == codes.tolist()
    assert (int(words[0]) & 0x0FFFFFFF) == 0x0FFFFFFF      # bases 0..13 untouched
    assert (int(words[1]) >> 6) == (0xFFFFFFFF >> 6)       # bases 19.. untouched


def test_null_context_is_rejected_without_touching_a_device(L):
    from paper_2002_05200_amd import xdrop
    sc = xdrop.Scores(1, -1, -1)
    rc = L.xdrop_extend(None, None, 0, None, 0, None, 1, sc, None, None, None)
    assert rc == xdrop.XD_EINVAL
    assert "null context" in xdrop.last_error()
    assert L.xd_last_stats(None, None) == xdrop.XD_EINVAL
    L.xd_ctx_destroy(None)


def test_struct_layouts_match_header(tmp_path):
    """The binding's structs have the sizes and field offsets a C compiler
    gives the header's structs."""
    import subprocess
    from paper_2002_05200_amd import xdrop
    structs = {"xd_pair": None, "xd_result": None, "xd_opts": xdrop.Opts,
               "xd_stats": xdrop.Stats, "xd_server_opts": xdrop.ServerOpts,
               "xd_request": xdrop.Request, "xd_server_stats": xdrop.ServerStats,
               "xd_seed": None}
    fields = {"xd_opts": [f for f, _ in xdrop.Opts._fields_],
              "xd_stats": [f for f, _ in xdrop.Stats._fields_],
              "xd_server_opts": [f for f, _ in xdrop.ServerOpts._fields_],
              "xd_pair": list(xdrop.PAIR_DTYPE.names),
              "xd_seed": list(xdrop.SEED_DTYPE.names),
              "xd_result": list(xdrop.RESULT_DTYPE.names)}
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "xdrop.h"', "int main(void) {"]
    for s in structs:
        src.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for f in fields.get(s, []):
            src.append(f'printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    src.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", f"-I{os.path.dirname(HEADER)}", str(c), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    assert int(got["xd_pair"]) == xdrop.PAIR_DTYPE.itemsize == 40
    assert int(got["xd_result"]) == xdrop.RESULT_DTYPE.itemsize == 56
    for name, dt in (("xd_pair", xdrop.PAIR_DTYPE), ("xd_result", xdrop.RESULT_DTYPE),
                     ("xd_seed", xdrop.SEED_DTYPE)):
        for f in dt.names:
            assert int(got[f"{name}.{f}"]) == dt.fields[f][1], (name, f)
    for s, cls in structs.items():
        if cls is None:
            continue
        assert int(got[s]) == ctypes.sizeof(cls), s
        for f in fields.get(s, []):
            assert int(got[f"{s}.{f}"]) == getattr(cls, f).offset, (s, f)
    text = open(HEADER).read()
    assert "} xd_opts; /* 48 bytes */" in text and int(got["xd_opts"]) == 48
    assert "} xd_server_opts; /* 80 bytes */" in text and int(got["xd_server_opts"]) == 80
    assert "} xd_seed; /* 32 bytes */" in text and int(got["xd_seed"]) == 32
    assert "} xd_request; /* 56 bytes */" in text and int(got["xd_request"]) == 56


def test_server_rejects_null_arguments_without_a_device(L):
    from paper_2002_05200_amd import xdrop
    assert L.xd_server_create(None, None) == xdrop.XD_EINVAL
    assert L.xd_server_submit(None, None, None) == xdrop.XD_EINVAL
    assert L.xd_server_poll(None, 1, None, 0, None) == xdrop.XD_EINVAL
    assert L.xd_server_get_stats(None, None) == xdrop.XD_EINVAL
    L.xd_server_destroy(None)


def test_noalloc_rejects_before_touching_a_device(L):
    """xdrop_extend_noalloc refuses oversize batches and the graph/profile
    options from the arguments alone (no device is touched, so this runs
    without a GPU; the pointers are never dereferenced)."""
    from paper_2002_05200_amd import xdrop
    fake = ctypes.c_void_p(0x1000)
    sc = xdrop.Scores(1, -1, -1)
    rc = L.xdrop_extend_noalloc(0, fake, 1, fake, 1, fake, xdrop.NOALLOC_MAX_PAIRS + 1, sc,
                                fake, None, None)
    assert rc == xdrop.XD_EINVAL and "XD_NOALLOC_MAX_PAIRS" in xdrop.last_error()
    for kw in (dict(profile=1), dict(graph=1)):
        o = xdrop.make_opts(**kw)
        rc = L.xdrop_extend_noalloc(0, fake, 1, fake, 1, fake, 4, sc, fake, fake, ctypes.byref(o))
        assert rc == xdrop.XD_EINVAL, kw
    rc = L.xdrop_extend_noalloc(0, fake, 1, fake, 1, fake, 4, xdrop.Scores(1, 2, -1), fake,
                                None, None)
    assert rc == xdrop.XD_EINVAL
    assert L.xdrop_extend_noalloc(0, None, 0, None, 0, None, 0, sc, None, None, None) == 0
    text = open(HEADER).read()
    assert re.search(r"#define XD_NOALLOC_MAX_PAIRS %d\b" % xdrop.NOALLOC_MAX_PAIRS, text)
