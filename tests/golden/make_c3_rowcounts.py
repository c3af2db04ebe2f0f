"""Writes c3_rowcounts.json: for every set of the clustered 32-set batch
(workloads.clustered_batch(), 5.6 million particles), the oracle's neighbour count of
every row, stored as the set's size, its total (nnz) and the SHA-256 of the counts as
little-endian int64 (the 5.6 million counts themselves would not fit a fixture).
Calls only the oracle (oracle.count_rows, the cell-list search with rows in parallel).

    python tests/golden/make_c3_rowcounts.py
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2401_08586_amd import workloads as W  # noqa: E402


def digest(counts):
    return hashlib.sha256(np.ascontiguousarray(counts, dtype="<i8").tobytes()).hexdigest()


def main():
    pss = W.clustered_batch()
    out = {"workload": "workloads.clustered_batch() (32 clustered 3D sets, seed 3)",
           "how": "oracle.count_rows per set; counts_sha256 = sha256 of the counts as little-endian int64",
           "sets": []}
    t0 = time.time()
    for s, ps in enumerate(pss):
        c = oracle.count_rows(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius)
        out["sets"].append({"set": s, "n": ps.n, "nnz": int(c.sum()), "max_row": int(c.max()),
                            "counts_sha256": digest(c)})
        print(f"set {s}: n={ps.n} nnz={int(c.sum())} ({time.time() - t0:.0f} s)", flush=True)
    out["nnz_total"] = sum(e["nnz"] for e in out["sets"])
    with open(os.path.join(HERE, "c3_rowcounts.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
