"""Write seqgen_manifest.txt: for every synthetic workload at seed 0, its
pair count, base count and the SHA-256 of its arrays (seqgen's
PairBatch.digest). The manifest pins the generator, so a benchmark figure
always refers to the same inputs; tests/test_abi.py regenerates and compares.

    python tests/golden/make_manifest.py
"""

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import seqgen  # noqa: E402


def main():
    lines = ["# workload pairs bases sha256 (seqgen.make_workload(workload), seed 0)"]
    for name in seqgen.WORKLOADS:
        b = seqgen.make_workload(name)
        lines.append(f"{name} {b.n_pairs} {int(b.t_len.sum() + b.q_len.sum())} {b.digest()}")
    with open(os.path.join(HERE, "seqgen_manifest.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
