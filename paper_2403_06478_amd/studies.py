"""Sensitivity studies of Sections 5.5-5.7, redone for the wave64 kernels.

Every study runs synthetic batches (``seqgen``) through ``ga_align_batch``
and prints one JSON line per point; results must be identical across the
variants of a point (the study stops otherwise).

* ``long_ratio`` (Section 5.6, Fig. 12): batches mixing 4096-base and
  128-base pairs at a range of long-pair fractions, under the three
  schedules: ``unordered`` (persistent launches, pairs in batch order: the
  paper's original order), ``persistent`` (longest first: the counterpart
  of uneven bucketing) and ``bucketed`` (plain per-length-bucket launches).
* ``slots`` (Section 5.5's slice width has no counterpart here: every
  anti-diagonal's maximum is reduced in registers and tested one step
  later, so there is neither a slice of intermediate maxima in memory nor a
  run-ahead to trade; the kernel shape's own trade-off is the number of
  diagonals each lane holds): one batch per band width, forced onto each
  single-wave fixed class that holds the band (4 to 32 slots per lane).
* ``waves`` (Section 5.7's subwarp size, i.e. lanes per alignment): wide
  bands forced onto every class shape that holds them, one wave of 24 or 32
  slots per lane against 2-4 waves per pair.

``python -m paper_2403_06478_amd.studies [--study NAME ...]``
"""

from __future__ import annotations

import argparse
import json
import sys
from typing import List, Optional

import numpy as np

from . import CLASSES, Context, _torch, count_cells, ga_align_batch, ga_pair_class_in, pack_batch


def _log(msg: str):
    sys.stderr.write(f"[studies] {msg}\n")
    sys.stderr.flush()


def _run(ctx: Context, packed, batch, repeats: int):
    """(results, mean ms per call) of ga_align_batch on the current stream."""
    torch = _torch()
    out = ga_align_batch(ctx, packed, batch.scoring, batch.w, batch.zdrop)
    torch.cuda.synchronize()
    ctx.check()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(repeats):
        ga_align_batch(ctx, packed, batch.scoring, batch.w, batch.zdrop, out=out)
    ev1.record()
    torch.cuda.synchronize()
    ctx.check()
    return out.cpu().numpy(), ev0.elapsed_time(ev1) / repeats


def long_ratio(n_pairs: int = 100_000, fracs=(0.0, 0.001, 0.01, 0.05, 0.10, 0.25, 0.5, 1.0),
               bands=(751, 100), repeats: int = 3, device: int = 0):
    import seqgen
    ctx = Context(device)
    for w in bands:
        for f in fracs:
            b = seqgen.long_ratio(n_pairs, f, w=w)
            packed = pack_batch(ctx, b)
            line = {"study": "long_ratio", "pairs": n_pairs, "frac_long": f, "w": w, "Z": b.zdrop}
            ref = None
            cells = None
            for sched in ("unordered", "persistent", "bucketed"):
                ctx.set_schedule(sched)
                res, ms = _run(ctx, packed, b, repeats)
                if ref is None:
                    ref = res
                    cells = int(count_cells(b.t_len, b.q_len, w, res).sum())
                elif not np.array_equal(res, ref):
                    raise SystemExit(f"long_ratio w={w} f={f}: {sched} results differ")
                line[f"{sched}_ms"] = round(ms, 3)
                line[f"{sched}_gcups"] = round(cells / ms / 1e6, 1)
            ctx.set_schedule("persistent")
            line["cells"] = cells
            line["speedup_persistent"] = round(line["unordered_ms"] / line["persistent_ms"], 3)
            line["speedup_bucketed"] = round(line["unordered_ms"] / line["bucketed_ms"], 3)
            print(json.dumps(line), flush=True)
            _log(f"long_ratio w={w} f={f}: done")
    ctx.close()


def _shape_sweep(study: str, classes: List[int], bands, n_pairs: int, length: int, repeats: int,
                 device: int):
    import seqgen
    ctx = Context(device)
    rng = np.random.default_rng([7, length])
    base = seqgen.random_pairs(rng, n_pairs, length, length, err=0.05, w=-1, zdrop=400, name=study)
    for w in bands:
        b = seqgen.PairBatch(base.t_seq, base.t_off, base.t_len, base.q_seq, base.q_off, base.q_len,
                             dict(base.scoring), int(w), base.zdrop, f"{study}[w={w}]")
        packed = pack_batch(ctx, b)
        ctx.set_classes(None)
        default_cls = sorted({ga_pair_class_in(n, m, w, range(len(CLASSES)))
                              for n, m in zip(b.t_len.tolist(), b.q_len.tolist())})
        ref, ms = _run(ctx, packed, b, repeats)
        cells = int(count_cells(b.t_len, b.q_len, w, ref).sum())
        line = {"study": study, "pairs": n_pairs, "length": length, "w": w, "Z": b.zdrop, "cells": cells,
                "default_classes": [_shape(c) for c in default_cls], "default_ms": round(ms, 3),
                "default_gcups": round(cells / ms / 1e6, 1), "shapes": {}}
        for c in classes:
            if any(ga_pair_class_in(n, m, w, [c]) != c for n, m in zip(b.t_len.tolist(), b.q_len.tolist())):
                continue  # this shape does not hold every pair of the batch
            ctx.set_classes([c])
            res, ms = _run(ctx, packed, b, repeats)
            if not np.array_equal(res, ref):
                raise SystemExit(f"{study} w={w}: class {c} results differ")
            line["shapes"][_shape(c)] = {"ms": round(ms, 3), "gcups": round(cells / ms / 1e6, 1)}
        ctx.set_classes(None)
        print(json.dumps(line), flush=True)
        _log(f"{study} w={w}: done")
    ctx.close()


def _shape(c: int) -> str:
    k, nw, sl = CLASSES[c]
    return f"K{k}x{nw}" + ("s" if sl else "")


def slots(n_pairs: int = 20_000, length: int = 3000, bands=(50, 100, 200, 400, 751, 1000), repeats: int = 3,
          device: int = 0):
    fixed_one_wave = [c for c, (k, nw, sl) in enumerate(CLASSES) if nw == 1 and not sl]
    _shape_sweep("slots", fixed_one_wave, bands, n_pairs, length, repeats, device)


def waves(n_pairs: int = 6000, length: int = 8000, bands=(751, 900, 1200, 1500, 2000, 2500, 3500),
          repeats: int = 3, device: int = 0):
    wide = [c for c, (k, nw, sl) in enumerate(CLASSES) if k >= 24 and not sl]
    _shape_sweep("waves", wide, bands, n_pairs, length, repeats, device)


STUDIES = {"long_ratio": long_ratio, "slots": slots, "waves": waves}


def main(argv: Optional[list] = None):
    ap = argparse.ArgumentParser(description="kernel sensitivity studies (synthetic inputs)")
    ap.add_argument("--study", nargs="+", choices=sorted(STUDIES), default=["long_ratio", "slots", "waves"])
    ap.add_argument("--repeats", type=int, default=3)
    args = ap.parse_args(argv)
    torch = _torch()
    torch.cuda.set_device(0)
    for name in args.study:
        STUDIES[name](repeats=args.repeats)


if __name__ == "__main__":
    main()
