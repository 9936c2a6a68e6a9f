"""CPU-side checks of the C ABI library: it loads, exports every function the
public headers declare, and rejects bad arguments before touching a device.
No compute calls are made here."""
import ctypes
import glob
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1302_5507_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(soap_dp_\w+)\s*\(", text))
    return names


def test_library_built_and_exports_declared_symbols():
    assert os.path.exists(binding.LIB_PATH), "build with python -m paper_1302_5507_amd.build"
    declared = _declared()
    assert declared, "no declarations found"
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\b(soap_dp_\w+)\b", out))
    assert declared <= exported, declared - exported
    lib = binding.lib()
    for name in declared:
        assert hasattr(lib, name)
    assert set(binding.EXPORTED) <= declared


def test_library_contains_gfx950_code():
    # the offload bundle embedded by hipcc names its target
    data = open(binding.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_strerror_and_null_arguments():
    lib = binding.lib()
    assert binding.soap_dp_strerror(0) == "ok"
    for code in (-1, -2, -3, -4, -5, -6):
        assert binding.soap_dp_strerror(code) != "unknown error"
    assert lib.soap_dp_align_batch(None, None, None, None, None, 0) == binding.SOAP_DP_EINVAL
    assert (lib.soap_dp_align_batch_noalloc(None, None, None, None, None, 0)
            == binding.SOAP_DP_EINVAL)
    assert lib.soap_dp_create(None, 0) == binding.SOAP_DP_EINVAL
    assert lib.soap_dp_destroy(None) == binding.SOAP_DP_EINVAL
    assert binding.soap_dp_workspace_bytes(None, 10, 100, 250, 0) == 0
    assert lib.soap_dp_reserve(None, 10, 100, 250, 0) == binding.SOAP_DP_EINVAL
    assert binding.soap_dp_last_hip_error(None) == 0


def _unpack(words, count):
    w = np.asarray(words, dtype=np.uint32)
    k = np.arange(count)
    return ((w[k // 16] >> (2 * (k % 16)).astype(np.uint32)) & 3).astype(np.uint8)


def test_pack_words_roundtrip():
    rng = np.random.default_rng(0)
    for n in (0, 1, 15, 16, 17, 1000):
        codes = rng.integers(0, 4, size=n).astype(np.uint8)
        words = binding.pack_words(codes)
        assert words.size == (n + 15) // 16
        assert np.array_equal(_unpack(words, n), codes)
    # base k of a word sits in bits [2k, 2k+2)
    assert binding.pack_words(np.array([1, 2, 3], np.uint8))[0] == 1 | 2 << 2 | 3 << 4


def test_pack_reads_word_aligned():
    rng = np.random.default_rng(1)
    lens = np.array([5, 16, 17, 0, 33, 1])
    offs = np.concatenate([[0], np.cumsum(lens)[:-1]])
    codes = rng.integers(0, 4, size=int(lens.sum())).astype(np.uint8)
    words, woff = binding.pack_reads(codes, offs, lens)
    assert list(woff) == [0, 1, 2, 4, 4, 7]
    for t in range(len(lens)):
        got = _unpack(words[int(woff[t]):], int(lens[t]))
        assert np.array_equal(got, codes[offs[t]:offs[t] + lens[t]])


def test_pack_reads_interleaved():
    """Reads stored word by word in groups of 32: word k of read t at
    word_off[t] + 32 k, every read's bases intact, groups back to back."""
    rng = np.random.default_rng(2)
    lens = rng.integers(0, 90, size=101)
    offs = np.concatenate([[0], np.cumsum(lens)[:-1]])
    codes = rng.integers(0, 4, size=int(lens.sum())).astype(np.uint8)
    words, woff = binding.pack_reads_interleaved(codes, offs, lens)
    for t in range(len(lens)):
        k = np.arange(int(lens[t]))
        got = (words[int(woff[t]) + 32 * (k // 16)] >> (2 * (k % 16)).astype(np.uint32)) & 3
        assert np.array_equal(got.astype(np.uint8), codes[offs[t]:offs[t] + lens[t]])
    assert list(woff[:33] % 32) == list(range(32)) + [0]
    nw = (lens + 15) // 16
    assert words.size == sum(32 * int(nw[g:g + 32].max()) for g in range(0, len(lens), 32))


def test_ctypes_structs_match_header_layout(tmp_path):
    """Every ctypes mirror has the size and field offsets the C compiler gives
    the header's struct."""
    from paper_1302_5507_amd import serving
    pairs = {
        "soap_dp_scoring": binding.Scoring, "soap_dp_batch": binding.Batch,
        "soap_dp_result": binding.Result, "soap_dp_class_info": binding.ClassInfo,
        "soap_dp_multi_batch": binding.MultiBatch, "soap_dp_multi_result": binding.MultiResultABI,
        "soap_dp_mate_batch": binding.MateBatch, "soap_dp_mate_result": binding.MateResultABI,
        "soap_dp_server_config": serving.ServerConfig, "soap_dp_host_result": serving.HostResult,
        "soap_dp_request": serving.RequestStruct, "soap_dp_server_stats": serving.ServerStats,
    }
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "soap_dp.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n"):
        if line:
            c, f, v = line.split()
            got[(c, f)] = int(v)
    for cname, py in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


def test_server_rejects_bad_slot_counts_and_flags():
    """Argument checks of soap_dp_server_create run before any device call:
    1..8 slots, and align_flags 0 or SOAP_DP_FULL_WINDOW."""
    import ctypes
    from paper_1302_5507_amd import serving
    L = serving._lib()
    for n, flags in ((0, 0), (9, 0), (16, 0), (2, binding.BATCHED), (2, binding.SCORE_ONLY),
                     (2, 16)):
        cfg = serving.ServerConfig(0, n, 1024, 1024 * 16, 250, 410, binding.Scoring(1, -3, -5, -2),
                                   ctypes.c_void_p(64), 1, 0, 0, flags)
        h = ctypes.c_void_p()
        assert L.soap_dp_server_create(ctypes.byref(h), ctypes.byref(cfg)) == binding.SOAP_DP_EINVAL
        assert not h.value
