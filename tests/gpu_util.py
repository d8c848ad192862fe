"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
the oracle on the same seeded inputs, and compare element by element."""

from __future__ import annotations

import numpy as np

import oracle
import paper_2403_06478_amd as ga

_CTX = None
_TUNED = None
_WORKLOADS = {}


def context():
    global _CTX
    if _CTX is None:
        _CTX = ga.Context(0)
    return _CTX


def tuned_context():
    """A context with the autotuned class order, as the benchmark runs."""
    global _TUNED
    if _TUNED is None:
        _TUNED = ga.Context(0)
        _TUNED.autotune()
    return _TUNED


def workload(name):
    """A full synthetic workload at seed 0, drawn once per test process."""
    import seqgen
    if name not in _WORKLOADS:
        _WORKLOADS[name] = seqgen.make_workload(name)
    return _WORKLOADS[name]


def gpu_align(batch, w=None, Z=None, scoring=None, ctx=None):
    import torch
    ctx = ctx or context()
    packed = ga.pack_batch(ctx, batch)
    out = ga.ga_align_batch(ctx, packed, scoring or batch.scoring,
                            batch.w if w is None else w, batch.zdrop if Z is None else Z)
    torch.cuda.synchronize()
    ctx.check()
    return out.cpu().numpy()


def oracle_align(batch, w=None, Z=None, scoring=None, nthreads=None):
    out, cells = oracle.align_batch(batch, nthreads=nthreads, w=w, Z=Z, sc=scoring)
    return out, cells


def assert_same(got: np.ndarray, want: np.ndarray, batch=None, label=""):
    """Bit-exact comparison of [n, 7] int32 results, naming the first pairs
    that differ."""
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, (got.shape, want.shape)
    bad = np.nonzero(np.any(got != want, axis=1))[0]
    if bad.size:
        lines = [f"{label}: {bad.size} of {got.shape[0]} pairs differ"]
        for p in bad[:8]:
            extra = ""
            if batch is not None:
                extra = f" n={int(batch.t_len[p])} m={int(batch.q_len[p])}"
            lines.append(f"  pair {p}{extra}: gpu={got[p].tolist()} oracle={want[p].tolist()}")
        raise AssertionError("\n".join(lines))
