"""Regression anchors: the oracle still reproduces the values that
tests/golden/make_golden.py wrote from it, and the workload defaults match
the constants fixture (Listing 1's M; the workloads' LCG and stride)."""
import json
import os

import workloads as W

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _constants():
    out = {}
    for line in open(os.path.join(GOLD, "paper_constants.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = int(v, 0)
    return out


def test_constants_fixture(orc):
    c = _constants()
    lcg = W.Lcg()
    assert (lcg.g, lcg.c, lcg.m, W.STRIDE_Q) == (c["lcg_g"], c["lcg_c"], c["lcg_m"], c["stride_q"])
    m = c["murmur_m"]
    # subhash(1) = M ^ (M >> shift) straight from Listing 1's first function
    assert orc.subhash(1) == m ^ (m >> c["murmur_shift"])
    assert orc.hash64(0, (c["murmur_len_factor"] * m) % (1 << 64)) == 0


def test_oracle_vectors_unchanged(orc):
    g = json.load(open(os.path.join(GOLD, "oracle_vectors.json")))
    lcg = W.Lcg()
    for k, s, h in g["hash"]:
        assert orc.hash64(k, s) == h
    for i, x in g["stride_start"]:
        assert orc.stream_start(lcg, W.stride_seeding(), i) == x
    for i, x in g["hash_start"]:
        assert orc.stream_start(lcg, W.hash_seeding(), i) == x
    for u, r in g["ln"]:
        assert orc.ln(float.fromhex(u)) == float.fromhex(r)
    for kind, sd in (("hash", W.hash_seeding()), ("stride", W.stride_seeding())):
        t = orc.transport(W.small_slab(sd), lcg)
        assert [hex(v) for v in t.raw] == g["small_slab_" + kind]["raw"]
        assert t.diag == g["small_slab_" + kind]["diag"]
