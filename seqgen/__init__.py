"""Seeded synthetic read-pair workloads.

This module only draws random sequences. It holds none of the alignment
arithmetic: it is shared by the oracle tests and the HIP path, and neither of
them imports the other.

The paper measures on Genome-in-a-Bottle HiFi/CLR/ONT reads mapped to GRCh38
after Minimap2 seeding and chaining (Section 5.1); none of that data is
available, so seeded synthetic pairs with the shapes of those workloads stand
in for it. Every sequence is ASCII (``A C G T`` and ``N``), concatenated into
one ``uint8`` buffer per side with ``int64`` start offsets and ``int32``
lengths, so the same bytes feed the oracle and the device packer.

Workload recipes (target = reference, query = mutated target), by name
(``make_workload(name)``; the number in brackets seeds the generator):

* ``uniform`` [1]  500 pairs, target length U{100..1000}, 5% errors
  (subst:ins:del 2:1:1), no N; band 500, z-drop 400.
* ``ont`` [2]  100k ONT-like pairs, target length clip(round(LogNormal(ln
  2000, 0.8)), 1, 20000), 10% errors (1:1:1), then every base of both
  sequences becomes N with probability 0.001; band 751, z-drop 400.
* ``mix`` [3]  1M pairs, target length min(50000, floor(50 * U**(-1/1.5)))
  (Pareto tail, alpha 1.5), 8% errors (1:1:1); 20% of the pairs get an
  unrelated U{2000..5000} random segment inserted into the query at a uniform
  position; band 751, z-drop 400.
* ``longread`` [4]  20k HiFi-like pairs, target length U{10000..25000}, 1%
  errors (1:1:1) plus U{1,2,3} long indels of U{50..500} bases each
  (insertion of random bases or deletion, probability 1/2 each); band 2000,
  z-drop 5000.
* ``serving`` [5]  serving requests, one pair each, in request order: with
  probability 0.95 drawn as in ``uniform``, else as in ``longread``; band
  500, z-drop 400 for every request. Arrival times are drawn by the serving
  benchmark.

``long_ratio`` (the synthetic study of Section 5.6, Fig. 12): a given
fraction of 4096-base targets among 128-base ones, 5% errors (1:1:1).

Point errors: each target base independently is an error with the stated
rate; a substitution draws one of the three other bases uniformly, an
insertion emits a random base after the original, a deletion drops the base.
Every workload is drawn from ``numpy.random.default_rng([number, seed])``.
"""

from __future__ import annotations

import dataclasses
import hashlib
from typing import Optional, Sequence

import numpy as np

ALPHABET = np.frombuffer(b"ACGT", dtype=np.uint8)
N_BYTE = ord("N")

# Scoring shared by every workload: match +2, mismatch -4, gap pieces
# (open 4, extend 2) and (open 24, extend 1), N scored -1.
SCORING = dict(a=2, b=4, q=4, e=2, q2=24, e2=1, ambig=1)


@dataclasses.dataclass
class PairBatch:
    """A batch of (target, query) pairs as concatenated ASCII buffers."""

    t_seq: np.ndarray  # uint8, concatenated targets
    t_off: np.ndarray  # int64, start of each target in t_seq
    t_len: np.ndarray  # int32
    q_seq: np.ndarray  # uint8, concatenated queries
    q_off: np.ndarray  # int64
    q_len: np.ndarray  # int32
    scoring: dict
    w: int
    zdrop: int
    name: str = "custom"

    @property
    def n_pairs(self) -> int:
        return int(self.t_len.shape[0])

    def target(self, p: int) -> bytes:
        o = int(self.t_off[p])
        return self.t_seq[o:o + int(self.t_len[p])].tobytes()

    def query(self, p: int) -> bytes:
        o = int(self.q_off[p])
        return self.q_seq[o:o + int(self.q_len[p])].tobytes()

    def subset(self, idx: Sequence[int]) -> "PairBatch":
        """A new batch holding pairs ``idx`` (in that order), re-concatenated."""
        idx = np.asarray(idx, dtype=np.int64)
        ts = [self.target(int(p)) for p in idx]
        qs = [self.query(int(p)) for p in idx]
        return from_lists(ts, qs, self.scoring, self.w, self.zdrop,
                          name=f"{self.name}[{len(idx)}]")

    def digest(self) -> str:
        h = hashlib.sha256()
        for arr in (self.t_seq, self.t_off, self.t_len, self.q_seq, self.q_off, self.q_len):
            h.update(np.ascontiguousarray(arr).tobytes())
        return h.hexdigest()


def from_lists(targets: Sequence[bytes], queries: Sequence[bytes], scoring: Optional[dict] = None,
               w: int = -1, zdrop: int = -1, name: str = "custom") -> PairBatch:
    """Build a batch from explicit byte strings (tests and examples)."""
    if len(targets) != len(queries):
        raise ValueError("targets and queries must have the same count")

    def pack(seqs):
        lens = np.array([len(s) for s in seqs], dtype=np.int32)
        off = np.zeros(len(seqs), dtype=np.int64)
        if len(seqs):
            off[1:] = np.cumsum(lens[:-1], dtype=np.int64)
        buf = np.frombuffer(b"".join(bytes(s) for s in seqs), dtype=np.uint8).copy()
        return buf, off, lens

    ts, to, tl = pack(targets)
    qs, qo, ql = pack(queries)
    return PairBatch(ts, to, tl, qs, qo, ql, dict(scoring or SCORING), int(w), int(zdrop), name)


def _random_bases(rng: np.random.Generator, count: int) -> np.ndarray:
    return ALPHABET[rng.integers(0, 4, size=count)]


def _mutate(rng: np.random.Generator, seq: np.ndarray, lens: np.ndarray, rate: float,
            ratio: Sequence[float]):
    """Apply per-base point errors to concatenated ``seq`` (segments ``lens``)."""
    L = seq.shape[0]
    kind = np.zeros(L, dtype=np.int8)  # 0 keep, 1 subst, 2 ins, 3 del
    err = rng.random(L) < rate
    p = np.asarray(ratio, dtype=np.float64)
    kind[err] = rng.choice(3, size=int(err.sum()), p=p / p.sum()).astype(np.int8) + 1
    base = seq.copy()
    sub = kind == 1
    if sub.any():
        code = np.searchsorted(ALPHABET, base[sub])
        base[sub] = ALPHABET[(code + rng.integers(1, 4, size=int(sub.sum()))) % 4]
    cnt = np.ones(L, dtype=np.int64)
    cnt[kind == 3] = 0
    cnt[kind == 2] = 2
    out = np.repeat(base, cnt)
    last = np.cumsum(cnt) - 1
    ins = kind == 2
    out[last[ins]] = _random_bases(rng, int(ins.sum()))
    seg_start = np.zeros(len(lens), dtype=np.int64)
    if len(lens):
        seg_start[1:] = np.cumsum(lens[:-1], dtype=np.int64)
    csum = np.concatenate([[0], np.cumsum(cnt)])
    new_lens = (csum[seg_start + lens] - csum[seg_start]).astype(np.int64)
    return out, new_lens


def _offsets(lens: np.ndarray) -> np.ndarray:
    off = np.zeros(len(lens), dtype=np.int64)
    if len(lens):
        off[1:] = np.cumsum(lens[:-1], dtype=np.int64)
    return off


def _splice(rng, q_seq, q_lens, which, seg_lo, seg_hi, mode):
    """Insert random segments into (mode 'ins') or delete segments from
    (mode 'del') the queries flagged in ``which``; one event per flag."""
    q_off = _offsets(q_lens)
    pieces = []
    new_lens = q_lens.copy()
    cursor = 0
    for p in np.nonzero(which)[0]:
        o, ln = int(q_off[p]), int(q_lens[p])
        pieces.append(q_seq[cursor:o])
        cur = q_seq[o:o + ln]
        seg = int(rng.integers(seg_lo, seg_hi + 1))
        if mode == "ins":
            pos = int(rng.integers(0, ln + 1))
            cur = np.concatenate([cur[:pos], _random_bases(rng, seg), cur[pos:]])
        else:
            seg = min(seg, max(ln - 1, 0))
            pos = int(rng.integers(0, ln - seg + 1)) if ln - seg >= 0 else 0
            cur = np.concatenate([cur[:pos], cur[pos + seg:]])
        pieces.append(cur)
        new_lens[p] = cur.shape[0]
        cursor = o + ln
    pieces.append(q_seq[cursor:])
    return np.concatenate(pieces) if pieces else q_seq, new_lens


def _sprinkle_n(rng, seq, rate):
    if rate > 0:
        hit = rng.random(seq.shape[0]) < rate
        seq = seq.copy()
        seq[hit] = N_BYTE
    return seq


def _finish(t_seq, t_lens, q_seq, q_lens, w, zdrop, name):
    t_lens = np.asarray(t_lens, dtype=np.int32)
    q_lens = np.asarray(q_lens, dtype=np.int32)
    return PairBatch(np.ascontiguousarray(t_seq, dtype=np.uint8), _offsets(t_lens), t_lens,
                     np.ascontiguousarray(q_seq, dtype=np.uint8), _offsets(q_lens), q_lens,
                     dict(SCORING), int(w), int(zdrop), name)


# name -> (seed number, pairs, band, z-drop)
WORKLOADS = {
    "uniform": (1, 500, 500, 400),
    "ont": (2, 100_000, 751, 400),
    "mix": (3, 1_000_000, 751, 400),
    "longread": (4, 20_000, 2000, 5000),
    "serving": (5, 20_000, 500, 400),
}


def _uniform_pairs(rng, P):
    tl = rng.integers(100, 1001, size=P)
    t = _random_bases(rng, int(tl.sum()))
    q, ql = _mutate(rng, t, tl, 0.05, (2, 1, 1))
    return t, tl, q, ql


def _long_read_pairs(rng, P):
    tl = rng.integers(10000, 25001, size=P)
    t = _random_bases(rng, int(tl.sum()))
    q, ql = _mutate(rng, t, tl, 0.01, (1, 1, 1))
    n_events = rng.integers(1, 4, size=P)
    for k in range(3):
        which = n_events > k
        is_ins = rng.random(P) < 0.5
        q, ql = _splice(rng, q, ql, which & is_ins, 50, 500, "ins")
        q, ql = _splice(rng, q, ql, which & ~is_ins, 50, 500, "del")
    return t, tl, q, ql


def _interleave(parts, which):
    """Pairs in request order: request k comes from parts[which[k]], each
    part consumed in its own order."""
    seqs = {"t": [], "q": []}
    pos = [0] * len(parts)
    offs = []
    for t, tl, q, ql in parts:
        offs.append((_offsets(np.asarray(tl)), _offsets(np.asarray(ql))))
    tl_out, ql_out = [], []
    for k in which:
        t, tl, q, ql = parts[k]
        i = pos[k]
        pos[k] += 1
        to, qo = offs[k][0][i], offs[k][1][i]
        seqs["t"].append(t[to:to + tl[i]])
        seqs["q"].append(q[qo:qo + ql[i]])
        tl_out.append(int(tl[i]))
        ql_out.append(int(ql[i]))
    t_all = np.concatenate(seqs["t"]) if seqs["t"] else np.zeros(0, np.uint8)
    q_all = np.concatenate(seqs["q"]) if seqs["q"] else np.zeros(0, np.uint8)
    return t_all, np.array(tl_out), q_all, np.array(ql_out)


def make_workload(name: str, n_pairs: Optional[int] = None, seed: int = 0) -> PairBatch:
    """Draw the workload ``name`` (a key of ``WORKLOADS``). ``n_pairs``
    truncates the draw to a prefix-sized batch with the same distribution (a
    smaller sample)."""
    if name not in WORKLOADS:
        raise ValueError(f"unknown workload {name!r} (one of {sorted(WORKLOADS)})")
    number, pairs, w, zdrop = WORKLOADS[name]
    rng = np.random.default_rng([number, seed])
    P = pairs if n_pairs is None else int(n_pairs)
    label = name + ("" if n_pairs is None else f"[{P}]")
    if name == "uniform":
        t, tl, q, ql = _uniform_pairs(rng, P)
        return _finish(t, tl, q, ql, w, zdrop, label)
    if name == "serving":
        # 95% drawn like the uniform pairs, 5% long-read-sized, in a random
        # request order; band 500 and z-drop 400 shared by every request
        is_long = rng.random(P) < 0.05
        n_long = int(is_long.sum())
        short = _uniform_pairs(rng, P - n_long)
        long_ = _long_read_pairs(rng, n_long)
        t, tl, q, ql = _interleave([short, long_], is_long.astype(np.int64))
        return _finish(t, tl, q, ql, w, zdrop, label)
    if name == "ont":
        tl = np.clip(np.round(rng.lognormal(np.log(2000.0), 0.8, size=P)), 1, 20000).astype(np.int64)
        t = _random_bases(rng, int(tl.sum()))
        q, ql = _mutate(rng, t, tl, 0.10, (1, 1, 1))
        t = _sprinkle_n(rng, t, 0.001)
        q = _sprinkle_n(rng, q, 0.001)
        return _finish(t, tl, q, ql, w, zdrop, label)
    if name == "mix":
        u = rng.random(P)
        u = np.maximum(u, np.finfo(np.float64).tiny)
        tl = np.minimum(50000, np.floor(50.0 * u ** (-1.0 / 1.5))).astype(np.int64)
        t = _random_bases(rng, int(tl.sum()))
        q, ql = _mutate(rng, t, tl, 0.08, (1, 1, 1))
        which = rng.random(P) < 0.20
        q, ql = _splice(rng, q, ql, which, 2000, 5000, "ins")
        return _finish(t, tl, q, ql, w, zdrop, label)
    t, tl, q, ql = _long_read_pairs(rng, P)  # longread
    return _finish(t, tl, q, ql, w, zdrop, label)


def long_ratio(n_pairs: int, frac_long: float, seed: int = 0, long_len: int = 4096,
               short_len: int = 128, err: float = 0.05, w: int = 751, zdrop: int = 400) -> PairBatch:
    """The long-pair ratio workload: round(frac_long * n_pairs) pairs with a
    ``long_len``-base target, the rest ``short_len``, at random positions in
    the batch; queries carry ``err`` point errors (1:1:1). Drawn from
    ``numpy.random.default_rng([6, seed])``."""
    rng = np.random.default_rng([6, seed])
    n_long = int(round(frac_long * n_pairs))
    tl = np.full(n_pairs, short_len, dtype=np.int64)
    tl[rng.permutation(n_pairs)[:n_long]] = long_len
    t = _random_bases(rng, int(tl.sum()))
    q, ql = _mutate(rng, t, tl, err, (1, 1, 1))
    return _finish(t, tl, q, ql, w, zdrop, f"long_ratio[{n_pairs},{frac_long:g}]")


def random_pairs(rng: np.random.Generator, n_pairs: int, len_lo: int, len_hi: int,
                 err: float = 0.1, ratio=(1, 1, 1), n_rate: float = 0.0,
                 related: float = 1.0, scoring: Optional[dict] = None, w: int = -1,
                 zdrop: int = -1, name: str = "random") -> PairBatch:
    """Small random batches for tests: target lengths U{len_lo..len_hi};
    a fraction ``related`` of queries are mutated targets, the rest are drawn
    independently with the same length distribution."""
    tl = rng.integers(len_lo, len_hi + 1, size=n_pairs)
    t = _random_bases(rng, int(tl.sum()))
    q, ql = _mutate(rng, t, tl, err, ratio)
    unrelated = rng.random(n_pairs) >= related
    if unrelated.any():
        q_off = _offsets(ql)
        pieces, lens = [], ql.copy()
        for p in range(n_pairs):
            if unrelated[p]:
                ln = int(rng.integers(len_lo, len_hi + 1))
                pieces.append(_random_bases(rng, ln))
                lens[p] = ln
            else:
                pieces.append(q[q_off[p]:q_off[p] + ql[p]])
        q = np.concatenate(pieces) if pieces else q
        ql = lens
    t = _sprinkle_n(rng, t, n_rate)
    q = _sprinkle_n(rng, q, n_rate)
    b = _finish(t, tl, q, ql, w, zdrop, name)
    if scoring is not None:
        b.scoring = dict(scoring)
    return b
