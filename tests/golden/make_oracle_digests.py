"""Write oracle_digests.txt: for every synthetic workload at seed 0, the
oracle's int32 results over ALL its pairs, as one SHA-256 per chunk of
1000 pairs (the first 16 hex digits), plus the workload's total cell count
and number of z-dropped pairs.

Only the CPU oracle computes these values (its -O3 -march=native build of
the same source, on the host that runs this script); the GPU parity test
then runs each full workload through the HIP path in one call, as the
benchmark times it, and compares every chunk. Each workload line carries
the digest of its inputs (the seqgen manifest's), so a stale file is
detected rather than trusted.

    python tests/golden/make_oracle_digests.py [workload ...]

Roughly half an hour on 8 cores (the long-read batch is 1.3e12 cells).
"""

import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import seqgen  # noqa: E402

CHUNK = 1000
OUT = os.path.join(HERE, "oracle_digests.txt")


def chunk_digests(results: np.ndarray, chunk: int = CHUNK):
    """SHA-256 (16 hex digits) of each chunk of rows of an [n, 7] int32
    result array, as little-endian bytes."""
    res = np.ascontiguousarray(np.asarray(results, dtype="<i4"))
    return [hashlib.sha256(res[k:k + chunk].tobytes()).hexdigest()[:16]
            for k in range(0, res.shape[0], chunk)]


def read_digests(path: str = OUT):
    """{workload: dict(digest=..., pairs=..., chunk=..., cells=..., zdropped=..., chunks=[...])}"""
    table = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "workload":
                name = parts[1]
                kv = dict(zip(parts[2::2], parts[3::2]))
                table[name] = dict(digest=kv["inputs"], pairs=int(kv["pairs"]), chunk=int(kv["chunk"]),
                                   cells=int(kv["cells"]), zdropped=int(kv["zdropped"]), chunks=[])
            else:
                name, k, h = parts
                assert int(k) == len(table[name]["chunks"])
                table[name]["chunks"].append(h)
    return table


def main(names):
    oracle.build(force=True, native=True)
    old = read_digests() if os.path.exists(OUT) else {}
    blocks = {}
    for name in seqgen.WORKLOADS:
        if names and name not in names:
            continue
        t0 = time.time()
        b = seqgen.make_workload(name)
        print(f"{name}: {b.n_pairs} pairs generated in {time.time() - t0:.1f} s", flush=True)
        t0 = time.time()
        res, cells = oracle.align_batch(b, nthreads=os.cpu_count() or 1, native=True)
        dt = time.time() - t0
        print(f"{name}: oracle {dt:.1f} s, {int(cells.sum())} cells "
              f"({cells.sum() / dt / 1e9:.2f} GCUPS), {int(res[:, 6].sum())} z-dropped", flush=True)
        blocks[name] = dict(digest=b.digest(), pairs=b.n_pairs, chunk=CHUNK, cells=int(cells.sum()),
                            zdropped=int(res[:, 6].sum()), chunks=chunk_digests(res))
    for name, v in old.items():
        blocks.setdefault(name, v)
    lines = ["# Oracle results over every pair of each synthetic workload at seed 0",
             "# (tests/golden/make_oracle_digests.py; written by the CPU oracle only).",
             "# 'workload' lines: the inputs' SHA-256 (seqgen PairBatch.digest), pair count,",
             "# chunk size, total algorithmic cells and z-dropped pairs; then one line per",
             "# chunk: workload, chunk index, SHA-256[:16] of the chunk's int32 results",
             "# (7 per pair, little-endian, pairs in batch order)."]
    for name in seqgen.WORKLOADS:
        if name not in blocks:
            continue
        v = blocks[name]
        lines.append(f"workload {name} inputs {v['digest']} pairs {v['pairs']} chunk {v['chunk']} "
                     f"cells {v['cells']} zdropped {v['zdropped']}")
        lines += [f"{name} {k} {h}" for k, h in enumerate(v["chunks"])]
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main(sys.argv[1:])
