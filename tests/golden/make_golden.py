"""Writes tests/golden/oracle_vectors.json from the CPU oracle alone.

These values are regression anchors for the oracle (a change to its
arithmetic shows up here); they are not pins of the method.  Run from the
repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def main():
    lcg = W.Lcg()
    out = {
        "hash": [[k, s, oracle.hash64(k, s)] for k, s in
                 ((1, 1), (2, 1), (1 << 26, 1), (12345, 42), ((1 << 64) - 1, 7), (0, 0))],
        "stride_start": [[i, oracle.stream_start(lcg, W.stride_seeding(), i)]
                         for i in (0, 1, 2, 1000, (1 << 26) - 1, 200_000_000)],
        "hash_start": [[i, oracle.stream_start(lcg, W.hash_seeding(), i)]
                       for i in (0, 1, 2, 1000, (1 << 26) - 1, 200_000_000)],
        "ln": [[u.hex(), oracle.ln(u).hex()] for u in (2.0 ** -53, 0.125, 0.3, 0.5, 0.7, 0.75, 0.999)],
    }
    for kind, sd in (("hash", W.hash_seeding()), ("stride", W.stride_seeding())):
        t = oracle.transport(W.small_slab(sd), lcg)
        out["small_slab_" + kind] = {"raw": [hex(v) for v in t.raw], "diag": t.diag}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_vectors.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
