"""Command-line front end: align the i-th record of a reference FASTA file
with the i-th record of a query FASTA file (the artifact interface of the
paper's appendix: options -a -b -q -r -z -w, scores written to
``<out>/score.log`` and the kernel time to ``<out>/time.json``).

The files are read on the host; packing (ASCII to 2-bit codes and the N
bitmap) and alignment run on the GPU through the C ABI.

``python -m paper_2403_06478_amd.cli REF.fasta QUERY.fasta [-a 2 -b 4 -q 4 -r 2 -z 400 -w 751]``
"""

from __future__ import annotations

import argparse
import json
import os
import sys
from typing import List, Tuple

import numpy as np


def read_fasta(path: str) -> Tuple[List[str], List[bytes]]:
    """Records of a FASTA file: (names, sequences). A record starts at a line
    beginning with '>' and holds the following lines up to the next header,
    concatenated, with whitespace removed. Bytes are kept as they are (case
    folding and N mapping happen in the packer: anything outside ACGTacgt is
    N)."""
    names: List[str] = []
    seqs: List[bytes] = []
    cur: List[bytes] = []
    with open(path, "rb") as f:
        for line in f:
            line = line.strip()
            if not line:
                continue
            if line.startswith(b">"):
                if names:
                    seqs.append(b"".join(cur))
                names.append(line[1:].strip().decode("utf-8", "replace"))
                cur = []
            else:
                if not names:
                    raise ValueError(f"{path}: sequence data before the first '>' header")
                cur.append(b"".join(line.split()))
    if names:
        seqs.append(b"".join(cur))
    return names, seqs


def make_batch(ref_path: str, query_path: str, scoring: dict, w: int, Z: int):
    import seqgen
    rn, rs = read_fasta(ref_path)
    qn, qs = read_fasta(query_path)
    if len(rs) != len(qs):
        raise ValueError(f"{ref_path} has {len(rs)} records, {query_path} has {len(qs)}: "
                         "the files must hold the same number of sequences")
    return rn, qn, seqgen.from_lists(rs, qs, scoring, w, Z, name=os.path.basename(query_path))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description="banded two-piece affine-gap extension alignment with z-drop")
    ap.add_argument("reference", help="FASTA file of targets (reference strings)")
    ap.add_argument("query", help="FASTA file of queries, one per reference record")
    ap.add_argument("-a", type=int, default=2, help="match score")
    ap.add_argument("-b", type=int, default=4, help="mismatch penalty")
    ap.add_argument("-q", type=int, default=4, help="gap open penalty (first piece)")
    ap.add_argument("-r", type=int, default=2, help="gap extension penalty (first piece)")
    ap.add_argument("--q2", type=int, default=24, help="gap open penalty of the second piece")
    ap.add_argument("--r2", type=int, default=1, help="gap extension penalty of the second piece")
    ap.add_argument("--ambig", type=int, default=1, help="penalty of a position involving N")
    ap.add_argument("-z", type=int, default=400, help="termination (z-drop) threshold; negative disables")
    ap.add_argument("-w", type=int, default=751, help="band width; negative for no band")
    ap.add_argument("-o", "--output", default="output", help="output folder")
    ap.add_argument("--device", type=int, default=0)
    args = ap.parse_args(argv)

    from . import Context, _torch, count_cells, ga_align_batch, pack_batch
    scoring = dict(a=args.a, b=args.b, q=args.q, e=args.r, q2=args.q2, e2=args.r2, ambig=args.ambig)
    rn, qn, batch = make_batch(args.reference, args.query, scoring, args.w, args.z)
    torch = _torch()
    ctx = Context(args.device)
    stream = torch.cuda.current_stream(args.device)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(stream)
    packed = pack_batch(ctx, batch)  # host-to-device copies, then the packing kernel
    ev[1].record(stream)
    out = ga_align_batch(ctx, packed, batch.scoring, batch.w, batch.zdrop)
    ev[2].record(stream)
    torch.cuda.synchronize(args.device)
    ctx.check()
    res = out.cpu().numpy() if batch.n_pairs else np.zeros((0, 7), dtype=np.int32)
    pack_ms, ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    ctx.close()

    os.makedirs(args.output, exist_ok=True)
    with open(os.path.join(args.output, "score.log"), "w") as f:
        f.write("#ref\tquery\tscore\tref_end\tquery_end\tend_score\tref_stop\tquery_stop\tzdropped\n")
        for k in range(batch.n_pairs):
            r = res[k]
            f.write(f"{rn[k]}\t{qn[k]}\t{r[0]}\t{r[1]}\t{r[2]}\t{r[3]}\t{r[4]}\t{r[5]}\t{r[6]}\n")
    cells = int(count_cells(batch.t_len, batch.q_len, batch.w, res).sum()) if batch.n_pairs else 0
    with open(os.path.join(args.output, "time.json"), "w") as f:
        json.dump({"kernel_ms": round(ms, 3), "pack_ms": round(pack_ms, 3), "pairs": batch.n_pairs, "cells": cells,
                   "gcups": round(cells / ms / 1e6, 3) if ms > 0 else None,
                   "scoring": scoring, "w": args.w, "z": args.z}, f)
        f.write("\n")
    sys.stderr.write(f"{batch.n_pairs} pairs aligned in {ms:.3f} ms; results in {args.output}/score.log\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
