"""The device layout's per-thread steps, run on the CPU.

tests/layout_emu.cpp includes the same step functions the layout kernels
call (csrc/layout_ops.h) and runs them one thread after another, in a
shuffled order, with plain-memory stand-ins for the atomics and a stable sort
in place of the device's radix sort.  Its node tables must equal the host
builder's for every valid leaf list and order, the presence cells must be
clear afterwards, and each invalid list must stop with the expected error
code.  This pins the layout's logic without a GPU; tests/test_gpu_layout.py
runs the kernels themselves.

Bar: exact (integer tables and codes).
"""
import os
import struct
import subprocess

import numpy as np
import pytest

import paper_2101_08226_amd as lib
import workloads as w
from helpers import random_amr_leaves

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2101_08226_amd", "csrc")
MAX_LEVEL = 9
CTL_WORDS = 2 + 3 * (MAX_LEVEL + 1)
NONE = 2**64 - 1
# error codes of the layout (the high word of the first error word)
E_LEVEL, E_INDEX, E_DUP, E_INSIDE, E_GAP, E_NEST = 1, 2, 3, 4, 5, 6


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    d = tmp_path_factory.mktemp("layemu")
    exe = str(d / "layemu")
    subprocess.run(["g++", "-std=c++17", "-O2", "-D__device__=", "-D__host__=", "-I" + CSRC,
                    "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "layout_emu.cpp"),
                    "-o", exe], check=True)
    return exe, d


def run(emu, leaves, levels, seed):
    exe, d = emu
    lv = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 4))
    fin, fout = str(d / "in.bin"), str(d / "out.bin")
    with open(fin, "wb") as f:
        f.write(struct.pack("<qiI", len(lv), levels, seed))
        f.write(lv.tobytes())
    subprocess.run([exe, fin, fout], check=True)
    b = open(fout, "rb").read()
    o = 0
    ctl = np.frombuffer(b, np.uint64, CTL_WORDS, o)
    o += 8 * CTL_WORDS
    cap = struct.unpack_from("<q", b, o)[0]
    o += 8
    host = np.frombuffer(b, np.int32, 2 * cap, o).reshape(-1, 2)
    o += 8 * cap
    res = {"ctl": ctl, "host": host, "levels": None}
    if int(ctl[1]) == NONE:
        nl = struct.unpack_from("<i", b, o)[0]
        o += 4
        lvls = []
        for _ in range(nl):
            nn, ni = struct.unpack_from("<qq", b, o)
            o += 16
            t = {"n_nodes": nn, "n_int": ni}
            for k, dt, shape in (("nbr", np.int32, (nn, 27)), ("child", np.int32, (ni, 8)),
                                 ("parent", np.int32, (nn,)), ("coord", np.int32, (nn, 3)),
                                 ("out_base", np.int64, (nn,))):
                a = np.frombuffer(b, dt, int(np.prod(shape)), o).reshape(shape)
                o += a.nbytes
                t[k] = a
            lvls.append(t)
        res["levels"] = lvls
    res["dirty"] = struct.unpack_from("<q", b, o)[0]
    return res


def valid_cases():
    out = []
    for s in range(1, 7):
        lv, _ = random_amr_leaves(s, max_level=3 + s % 3, n_stars=1 + s % 3)
        out.append((f"random{s}", lv))
    for lev in (0, 1, 3):
        out.append((f"uniform{lev}", w.uniform_leaves(lev)))
    out.append(("binary_l6", lib.octo_host_adaptive_leaves(w.binary_polytrope_128(), 6, 1e-4)))
    return out


@pytest.mark.parametrize("name,leaves", valid_cases(), ids=[c[0] for c in valid_cases()])
def test_layout_steps_equal_host_builder(emu, name, leaves):
    lv = np.asarray(leaves, dtype=np.int32).reshape(-1, 4)
    rng = np.random.default_rng(len(lv))
    nl_host, _ = lib.octo_host_layout(lv)
    deepest = int(lv[:, 0].max())
    # two orders of the list (the output offsets follow it) and two sizes of
    # the presence cells (one spare level)
    for seed, levels in ((1, deepest + 1), (2, min(deepest + 2, MAX_LEVEL + 1))):
        lvp = lv[rng.permutation(len(lv))]
        host = [lib.octo_host_level_tables(lvp, l) for l in range(nl_host)]
        r = run(emu, lvp, levels, seed)
        assert r["dirty"] == 0, "presence cells left set"
        assert int(r["ctl"][1]) == NONE, hex(int(r["ctl"][1]))
        assert len(r["levels"]) == nl_host
        pos = 0
        for l, (d, h) in enumerate(zip(r["levels"], host)):
            assert (d["n_nodes"], d["n_int"]) == (h["n_nodes"], h["n_int"]), l
            for k in ("nbr", "child", "parent", "coord", "out_base"):
                assert np.array_equal(d[k], h[k]), (l, k)
            hs = r["host"][pos:pos + h["n_nodes"]]
            ni = h["n_int"]
            assert np.array_equal(hs[:ni, 0], h["int_child"]), (l, "int_child")
            assert np.array_equal(hs[ni:, 0], h["flags"][ni:]), (l, "flags")
            assert np.array_equal(hs[:, 1], h["parent"]), (l, "parent")
            # the record leaves start at the first sorted position of class 2
            c2 = int(r["ctl"][2 + 3 * l + 2])
            n_rec = c2 - pos if c2 != NONE else h["n_nodes"]
            assert n_rec == h["n_rec"], l
            pos += h["n_nodes"]
        assert pos == int(r["ctl"][0])


def invalid_cases():
    lv = np.asarray(random_amr_leaves(3, max_level=3)[0], dtype=np.int32)
    i = int(np.argmin(lv[:, 0]))
    L, x, y, z = (int(v) for v in lv[i])
    kids = np.array([[L + 1, 2 * x + a, 2 * y + b, 2 * z + c] for a in (0, 1) for b in (0, 1) for c in (0, 1)],
                    np.int32)
    u = np.asarray(w.uniform_leaves(1), dtype=np.int32)
    k1 = np.array([[2, a, b, c] for a in (0, 1) for b in (0, 1) for c in (0, 1)], np.int32)
    k2 = np.array([[3, 2 + a, 2 + b, 2 + c] for a in (0, 1) for b in (0, 1) for c in (0, 1)], np.int32)
    return [
        ("duplicate", np.vstack([lv, lv[5:6]]), 4, E_DUP),
        ("level", np.vstack([lv, [[4, 0, 0, 0]]]), 4, E_LEVEL),
        ("negative level", np.vstack([lv, [[-1, 0, 0, 0]]]), 4, E_LEVEL),
        ("index", np.vstack([lv, [[2, 4, 0, 0]]]), 4, E_INDEX),
        ("overlap", np.vstack([lv, kids]), 5, E_INSIDE),
        ("gap", np.delete(lv, 7, axis=0), 4, E_GAP),
        ("nesting", np.vstack([u[1:], k1[:-1], k2]), 4, E_NEST),
    ]


@pytest.mark.parametrize("name,leaves,levels,code", invalid_cases(), ids=[c[0] for c in invalid_cases()])
def test_layout_steps_reject_invalid_lists(emu, name, leaves, levels, code):
    with pytest.raises(lib.OctoError):
        lib.octo_host_layout(leaves)
    for seed in (1, 2):
        r = run(emu, leaves, levels, seed)
        assert r["dirty"] == 0, "presence cells left set"
        assert int(r["ctl"][1]) != NONE
        assert int(r["ctl"][1]) >> 32 == code, (name, int(r["ctl"][1]) >> 32)
