"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs, bit-exact on all seven int32 result fields."""

from __future__ import annotations

import ctypes
import os
import sys

import numpy as np
import pytest

import seqgen
from brute import band_cells
from gpu_util import assert_same, gpu_align, oracle_align, tuned_context, workload

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _say(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


def test_uniform_500_pairs_full():
    b = seqgen.make_workload("uniform")
    _say(f"uniform 500 pairs: {b.n_pairs} pairs w={b.w} Z={b.zdrop}")
    want, _ = oracle_align(b)
    assert_same(gpu_align(b), want, b, "uniform")


def test_golden_closed_forms_on_gpu():
    from test_oracle_pins import _golden_cases
    for c in _golden_cases():
        b = seqgen.from_lists([c["T"]], [c["Q"]], c["sc"], c["w"], c["Z"], name=c["name"])
        _say(f"golden {c['name']}")
        got = gpu_align(b)
        assert tuple(got[0]) == c["res"], (c["name"], got[0].tolist(), c["res"])


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_random_small_batches(seed):
    """Random scorings, bands (including 0, 1, unbanded), thresholds
    (including 0 and disabled), N bases, related and unrelated pairs,
    lengths 0..400 (several tiles of every slot count, ragged tails)."""
    rng = np.random.default_rng(100 + seed)
    for trial in range(6):
        q = int(rng.integers(0, 8))
        e = int(rng.integers(1, 4))
        sc = dict(a=int(rng.integers(1, 6)), b=int(rng.integers(1, 9)), q=q, e=e,
                  q2=q + int(rng.integers(0, 30)), e2=int(rng.integers(0, e + 1)),
                  ambig=int(rng.integers(0, 5)))
        w = int(rng.choice([-1, 0, 1, 2, 5, 31, 64, 100, 255, 300]))
        Z = int(rng.choice([-1, 0, 5, 40, 200]))
        b = seqgen.random_pairs(rng, 120, 0, 400, err=float(rng.choice([0.02, 0.1, 0.3])),
                                n_rate=float(rng.choice([0.0, 0.01, 0.2])),
                                related=float(rng.choice([0.3, 0.8, 1.0])), scoring=sc, w=w, zdrop=Z)
        _say(f"random seed={seed} trial={trial} sc={sc} w={w} Z={Z}")
        want, _ = oracle_align(b)
        assert_same(gpu_align(b), want, b, f"seed={seed} trial={trial}")


def test_edge_cases():
    sc = dict(seqgen.SCORING)
    T, Q = [], []
    cases = [(b"", b"ACGT"), (b"ACGT", b""), (b"", b""), (b"A", b"A"), (b"A", b"C"), (b"N", b"N"),
             (b"ACGTACGTAC" * 30, b"ACGTACGTAC" * 30), (b"N" * 200, b"N" * 150),
             (b"ACGT" * 100, b"ACG"), (b"A", b"ACGT" * 100), (b"ACGT" * 10, b"TGCA" * 200)]
    for t, q in cases:
        T.append(t)
        Q.append(q)
    for w in (-1, 0, 1, 2, 3, 7, 64, 500, 1023):
        for Z in (-1, 0, 3, 400):
            b = seqgen.from_lists(T, Q, sc, w, Z)
            want, _ = oracle_align(b)
            assert_same(gpu_align(b), want, b, f"edge w={w} Z={Z}")


def test_band_wider_than_sequences_and_lopsided():
    """|n-m| > w (band cuts the corner), n or m much shorter than w, and the
    largest band each slot count holds (2w+1 = 512, 1024, 1536, 2047)."""
    rng = np.random.default_rng(55)
    for w in (4, 30, 255, 511, 767, 1023):
        b = seqgen.random_pairs(rng, 40, 1, 1500, err=0.1, n_rate=0.005, related=0.8,
                                w=w, zdrop=int(rng.choice([-1, 100])))
        _say(f"lopsided w={w}")
        want, _ = oracle_align(b)
        assert_same(gpu_align(b), want, b, f"lopsided w={w}")


def test_ont_like_sample():
    b = seqgen.make_workload("ont", n_pairs=400)
    _say(f"ONT-like sample: {b.n_pairs} pairs")
    want, _ = oracle_align(b)
    assert_same(gpu_align(b), want, b, "ont[400]")


def test_mix_sample():
    full = seqgen.make_workload("mix", n_pairs=4000)
    # keep the oracle's work bounded: drop the rare >8 kb targets
    idx = np.nonzero(full.t_len <= 8000)[0][:1500]
    b = full.subset(idx)
    _say(f"mix sample: {b.n_pairs} pairs")
    want, _ = oracle_align(b)
    got = gpu_align(b)
    assert_same(got, want, b, "mix sample")
    # short targets cannot fall Z = 400 below their maximum, so only the
    # longer pairs with an inserted segment drop
    assert got[:, 6].sum() >= 1


@pytest.mark.parametrize("name", ["uniform", "ont", "mix", "longread", "serving"])
def test_full_workload_every_pair(name):
    """Every pair of each full synthetic workload, run in one call with the
    autotuned class order (as the benchmark times it), against the oracle's
    results stored as one SHA-256 per 1000-pair chunk
    (tests/golden/oracle_digests.txt, written on the CPU by
    make_oracle_digests.py beside it). A chunk that differs is re-aligned by
    the oracle here and its differing pairs are named."""
    import paper_2403_06478_amd as ga
    sys.path.insert(0, os.path.join(HERE, "golden"))
    from make_oracle_digests import chunk_digests, read_digests
    ref = read_digests()[name]
    b = workload(name)
    assert b.n_pairs == ref["pairs"] and b.digest() == ref["digest"], "inputs differ from the digests' inputs"
    _say(f"every pair of {name}: {b.n_pairs} pairs, w={b.w} Z={b.zdrop}")
    got = gpu_align(b, ctx=tuned_context())
    C = ref["chunk"]
    mine = chunk_digests(got, C)
    bad = [k for k, (x, y) in enumerate(zip(mine, ref["chunks"])) if x != y]
    if bad:
        k = bad[0]
        idx = np.arange(k * C, min(b.n_pairs, (k + 1) * C))
        sub = b.subset(idx)
        want, _ = oracle_align(sub)
        assert_same(got[idx], want, sub, f"{name}: {len(bad)} of {len(mine)} chunks differ; chunk {k}")
        raise AssertionError(f"{name}: chunk {k} digest differs but its pairs match the oracle run here")
    assert len(mine) == len(ref["chunks"])
    assert int(got[:, 6].sum()) == ref["zdropped"]
    cells = ga.count_cells(b.t_len, b.q_len, b.w, got)
    assert int(cells.sum()) == ref["cells"]
    _say(f"every pair of {name}: {len(mine)} chunks equal, {int(cells.sum())} cells, "
          f"{ref['zdropped']} z-dropped")


def test_ont_like_100k_full_size_sampled():
    """The bench workload at full size (100k pairs, one launch): sampled
    pairs against the oracle, every pair against cheap properties."""
    b = workload("ont")
    _say(f"ONT-like full: {b.n_pairs} pairs")
    got = gpu_align(b)
    rng = np.random.default_rng(2)
    idx = np.sort(rng.choice(b.n_pairs, size=120, replace=False))
    sub = b.subset(idx)
    want, _ = oracle_align(sub)
    assert_same(got[idx], want, sub, "ont full sampled")
    # properties at every pair: G >= 0, positions inside the matrix, the end
    # on an anti-diagonal no later than the last cell, the flag binary
    n, m = b.t_len.astype(np.int64), b.q_len.astype(np.int64)
    assert np.all(got[:, 0] >= 0)
    assert np.all((got[:, 1] >= -1) & (got[:, 1] < n) & (got[:, 2] >= -1) & (got[:, 2] < m))
    assert np.all((got[:, 4] >= 0) & (got[:, 4] < n) & (got[:, 5] >= 0) & (got[:, 5] < m))
    assert np.all(np.abs(got[:, 4] - got[:, 5]) <= b.w)
    assert set(np.unique(got[:, 6]).tolist()) <= {0, 1}
    assert np.all(got[:, 3] <= got[:, 0])  # the end is never above the maximum


def test_mix_1m_full_size_sampled():
    """The heavy-tailed 1M-pair workload in one call (every class, the
    streams overlapped, as timed): random pairs, the longest pairs, pairs
    that dropped and short-by-long pairs against the oracle; every pair
    against cheap properties."""
    import paper_2403_06478_amd as ga
    b = workload("mix")
    _say(f"mix full: {b.n_pairs} pairs")
    got = gpu_align(b)
    rng = np.random.default_rng(3)
    n, m = b.t_len.astype(np.int64), b.q_len.astype(np.int64)
    longest = np.argsort(-(n + m), kind="stable")[:4]
    dropped = np.nonzero(got[:, 6] == 1)[0]
    lopsided = np.nonzero(np.abs(m - n) > 2 * b.w)[0]
    idx = np.unique(np.concatenate([
        rng.choice(b.n_pairs, size=160, replace=False), longest,
        rng.choice(dropped, size=min(16, dropped.size), replace=False),
        rng.choice(lopsided, size=min(24, lopsided.size), replace=False)]))
    classes = {ga.class_name(ga.ga_pair_class(int(n[p]), int(m[p]), b.w)) for p in idx}
    _say(f"mix full: {idx.size} sampled pairs in classes {sorted(classes)}")
    assert any("sliding" in c for c in classes)
    sub = b.subset(idx)
    want, _ = oracle_align(sub)
    assert_same(got[idx], want, sub, "mix full sampled")
    assert np.all(got[:, 0] >= 0)
    assert np.all((got[:, 1] >= -1) & (got[:, 1] < n) & (got[:, 2] >= -1) & (got[:, 2] < m))
    assert np.all((got[:, 4] >= 0) & (got[:, 4] < n) & (got[:, 5] >= 0) & (got[:, 5] < m))
    assert np.all(np.abs(got[:, 4] - got[:, 5]) <= b.w)
    assert set(np.unique(got[:, 6]).tolist()) <= {0, 1}
    assert np.all(got[:, 3] <= got[:, 0])


def test_deterministic_and_order_independent():
    b = seqgen.make_workload("ont", n_pairs=300)
    x = gpu_align(b)
    y = gpu_align(b)
    assert np.array_equal(x, y)
    perm = np.random.default_rng(9).permutation(b.n_pairs)
    z = gpu_align(b.subset(perm))
    assert np.array_equal(z, x[perm])


def test_suffix_invariance_after_drop():
    """Bases beyond the termination anti-diagonal cannot change the result
    (no cell computed ahead of the termination test leaks into it)."""
    rng = np.random.default_rng(77)
    b = seqgen.random_pairs(rng, 200, 200, 900, err=0.1, related=0.3, w=200, zdrop=60)
    got = gpu_align(b)
    T, Q = [], []
    for p in range(b.n_pairs):
        t, q = bytearray(b.target(p)), bytearray(b.query(p))
        if got[p, 6]:
            r_end = int(got[p, 4] + got[p, 5])
            for s in (t, q):
                for k in range(r_end + 1, len(s)):
                    s[k] = ord("ACGTN"[(s[k] + 3 * k) % 5])
        T.append(bytes(t))
        Q.append(bytes(q))
    b2 = seqgen.from_lists(T, Q, b.scoring, b.w, b.zdrop)
    assert np.array_equal(gpu_align(b2), got)
    assert got[:, 6].sum() > 40


def test_unsupported_band_raises():
    """Bands of more than 8180 diagonals are refused before any launch."""
    import paper_2403_06478_amd as ga
    b = seqgen.random_pairs(np.random.default_rng(1), 4, 5000, 5000, w=4096, zdrop=5000)
    with pytest.raises(ga.GaError) as ei:
        gpu_align(b)
    assert ei.value.code == ga.GA_EUNSUPPORTED


@pytest.mark.parametrize("sc", [
    dict(a=27, b=228, q=60, e=20, q2=100, e2=5, ambig=228),  # every byte-table limit reached
    dict(a=127, b=128, q=0, e=0, q2=0, e2=0, ambig=128),     # free gaps, extreme substitution scores
    dict(a=1, b=0, q=0, e=1, q2=3, e2=0, ambig=0),           # free second piece: long gaps cost q2 only
])
def test_score_table_limits(sc):
    """Scorings at the limits of the per-cell score bytes (S + q + 2e in
    -128..127) and degenerate gap costs, bit-exact against the oracle with
    and without z-drop; one past a limit is refused before any launch."""
    import paper_2403_06478_amd as ga
    b = seqgen.random_pairs(np.random.default_rng(sc["a"] + sc["b"]), 60, 0, 500, err=0.15, n_rate=0.05,
                            related=0.7, scoring=sc, w=100, zdrop=200)
    for Z in (200, -1):
        want, _ = oracle_align(b, Z=Z, scoring=sc)
        assert_same(gpu_align(b, Z=Z, scoring=sc), want, b, f"score limits {sc} Z={Z}")
    fold = sc["q"] + 2 * sc["e"]
    for past in (dict(sc, a=127 - fold + 1), dict(sc, b=fold + 129), dict(sc, ambig=fold + 129)):
        with pytest.raises(ga.GaError) as ei:
            gpu_align(b, scoring=past)
        assert ei.value.code == ga.GA_EUNSUPPORTED


def test_scores_at_the_range_guard():
    """Two-million-base pairs with large scores, the range guard
    (2 max_len + 2) * (max(a, b, ambig, q+e, q2+e2) + a + e + e2) + Z
    < 2^29 filled to 97%: identical sequences, one with 1000 inserted bases
    and an unrelated pair, with and without z-drop, bit-exact against the
    oracle; one base more than the guard allows is refused before any
    launch."""
    import paper_2403_06478_amd as ga
    sc = dict(a=30, b=60, q=40, e=20, q2=70, e2=5, ambig=40)
    n, w = 2_000_000, 64
    rng = np.random.default_rng(77)
    acgt = np.frombuffer(b"ACGT", dtype=np.uint8)
    t = acgt[rng.integers(0, 4, size=n)].tobytes()
    ins = acgt[rng.integers(0, 4, size=1000)].tobytes()
    other = acgt[rng.integers(0, 4, size=n)].tobytes()
    b = seqgen.from_lists([t, t, t], [t, t[:n // 2] + ins + t[n // 2:], other], sc, w, 400)
    P = max(sc["a"], sc["b"], sc["ambig"], sc["q"] + sc["e"], sc["q2"] + sc["e2"])
    guard = (2 * (n + 1000) + 2) * (P + sc["a"] + sc["e"] + sc["e2"]) + 400
    assert 0.95 * 2 ** 29 < guard < 2 ** 29
    for Z in (400, -1):
        _say(f"range guard: 3 pairs of {n} bases, w={w}, Z={Z}")
        want, _ = oracle_align(b, Z=Z, scoring=sc)
        got = gpu_align(b, Z=Z, scoring=sc)
        assert_same(got, want, b, f"range guard Z={Z}")
        assert got[0, 0] == sc["a"] * n and got[0, 1] == n - 1 and got[0, 2] == n - 1
    k = P + sc["a"] + sc["e"] + sc["e2"]
    over = -(-(2 ** 29) // (2 * k)) - 1  # the shortest max_len the guard refuses at Z=0
    assert (2 * over + 2) * k >= 2 ** 29 > (2 * over) * k
    big = acgt[rng.integers(0, 4, size=over)].tobytes()
    with pytest.raises(ga.GaError) as ei:
        gpu_align(seqgen.from_lists([big], [big[:100]], sc, w, 0), Z=0, scoring=sc)
    assert ei.value.code == ga.GA_EINVAL


@pytest.mark.parametrize("w", [1024, 1100, 1533, 1534, 2045, 2046, 3067, 3068, 4089])
def test_multiwave_bands(w):
    """Bands wider than one wave holds (2w+1 > 2048 diagonals) run on 2-4
    waves per pair: the class boundaries (3068, 4092, 6136, 8180 diagonals),
    pairs shorter and longer than the band, unrelated pairs that z-drop,
    N bases, and lopsided lengths whose band is cut by the rectangle."""
    import paper_2403_06478_amd as ga
    rng = np.random.default_rng(4000 + w)
    lo = max(1, w - 300)
    b = seqgen.random_pairs(rng, 14, lo, w + 900, err=0.08, n_rate=0.005, related=0.7,
                            w=w, zdrop=int(rng.choice([-1, 150, 400])))
    cls = [ga.ga_pair_class(int(n), int(m), w) for n, m in zip(b.t_len, b.q_len)]
    _say(f"multiwave w={w} Z={b.zdrop}: classes {sorted(set(cls))}")
    assert max(cls) >= 5  # a multi-wave class
    want, _ = oracle_align(b)
    assert_same(gpu_align(b), want, b, f"multiwave w={w}")


def test_multiwave_unbanded_and_drops():
    """w < 0 with lengths whose n + m + 1 needs 2-4 waves, and small Z so the
    z-drop fires inside multi-wave sweeps at many different anti-diagonals."""
    rng = np.random.default_rng(77)
    sc = dict(seqgen.SCORING)
    for Z, related in ((-1, 1.0), (30, 0.5), (0, 0.3)):
        b = seqgen.random_pairs(rng, 10, 1100, 2600, err=0.1, n_rate=0.01, related=related,
                                scoring=sc, w=-1, zdrop=Z)
        _say(f"multiwave unbanded Z={Z}")
        want, _ = oracle_align(b)
        got = gpu_align(b)
        assert_same(got, want, b, f"unbanded Z={Z}")
        if Z >= 0:
            assert got[:, 6].sum() >= 1


def test_long_reads_sample():
    """The long-read workload (w=2000, Z=5000, 10-25 kb): a few whole pairs
    against the oracle."""
    b = seqgen.make_workload("longread", n_pairs=6)
    _say(f"long-read sample: {b.n_pairs} pairs, lengths {b.t_len.tolist()}")
    want, _ = oracle_align(b)
    assert_same(gpu_align(b), want, b, "longread[6]")


def test_long_reads_20k_full_size_sampled():
    """The whole 20k-pair long-read workload in one launch: sampled pairs
    against the oracle, every pair against cheap properties."""
    b = workload("longread")
    _say(f"long-read full: {b.n_pairs} pairs")
    got = gpu_align(b)
    rng = np.random.default_rng(4)
    idx = np.sort(rng.choice(b.n_pairs, size=8, replace=False))
    sub = b.subset(idx)
    want, _ = oracle_align(sub)
    assert_same(got[idx], want, sub, "longread full sampled")
    n, m = b.t_len.astype(np.int64), b.q_len.astype(np.int64)
    assert np.all(got[:, 0] >= 0)
    assert np.all((got[:, 4] >= 0) & (got[:, 4] < n) & (got[:, 5] >= 0) & (got[:, 5] < m))
    assert np.all(np.abs(got[:, 4] - got[:, 5]) <= b.w)
    assert set(np.unique(got[:, 6]).tolist()) <= {0, 1}
    assert np.all(got[:, 3] <= got[:, 0])


def test_cells_closed_form():
    import paper_2403_06478_amd as ga
    b = seqgen.make_workload("uniform", n_pairs=60)
    got = gpu_align(b)
    _, cells = oracle_align(b)
    lib_cells = ga.count_cells(b.t_len, b.q_len, b.w, got)
    assert np.array_equal(lib_cells, cells)


def test_planner_writes_every_pair_once():
    """The cost-ordered work lists cover every pair exactly once: many pairs
    share a cost bucket (equal lengths), others are alone in theirs, the
    classes mix, and the output starts as a sentinel that no result equals."""
    import torch

    import paper_2403_06478_amd as ga
    from gpu_util import context
    rng = np.random.default_rng(31)
    same = seqgen.random_pairs(rng, 300, 700, 700, err=0.05, related=1.0, w=600, zdrop=400)
    mixed = seqgen.random_pairs(rng, 300, 0, 2600, err=0.1, n_rate=0.01, related=0.7, w=600, zdrop=400)
    T = [same.target(p) for p in range(same.n_pairs)] + [mixed.target(p) for p in range(mixed.n_pairs)]
    Q = [same.query(p) for p in range(same.n_pairs)] + [mixed.query(p) for p in range(mixed.n_pairs)]
    order = rng.permutation(len(T))
    b = seqgen.from_lists([T[k] for k in order], [Q[k] for k in order], seqgen.SCORING, 600, 400)
    _say(f"planner: {b.n_pairs} pairs, classes "
         f"{np.bincount([ga.ga_pair_class(int(n), int(m), 600) + 1 for n, m in zip(b.t_len, b.q_len)])}")
    ctx = context()
    packed = ga.pack_batch(ctx, b)
    out = torch.full((b.n_pairs, 7), -777, dtype=torch.int32, device="cuda")
    for _ in range(2):  # twice: the second call reuses the workspace
        ga.ga_align_batch(ctx, packed, b.scoring, b.w, b.zdrop, out=out)
        torch.cuda.synchronize()
        ctx.check()
        got = out.cpu().numpy()
        assert not np.any(got == -777)
        want, _ = oracle_align(b)
        assert_same(got, want, b, "planner")
        out.fill_(-777)


def test_valu_calibration_plausible():
    """The VALU probe measures between a quarter of and a little above the
    published int32 lane-op peak (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz);
    the box has measured about 4% above it."""
    from gpu_util import context
    v = context().calibrate_valu() / 1e12
    _say(f"measured int32 VALU peak {v:.2f} T lane-ops/s")
    assert 0.25 * 39.32 < v < 1.15 * 39.32


def test_boundary_cells_never_counted():
    """Near the origin the boundary cells (-1, r+1) and (r+1, -1) can score
    above every cell of their anti-diagonal (heavy mismatch penalty, cheap
    long gaps); they must never become the anti-diagonal maximum. All-mismatch
    and unrelated pairs over several bands, scorings and thresholds."""
    rng = np.random.default_rng(606)
    T, Q = [], []
    for k in range(60):
        n, m = int(rng.integers(2, 300)), int(rng.integers(2, 300))
        if k % 3 == 0:
            t, q = b"A" * n, b"C" * m
        else:
            t = bytes(rng.choice(list(b"ACGT"), n))
            q = bytes(rng.choice(list(b"ACGT"), m))
        T.append(t)
        Q.append(q)
    for sc in (dict(a=1, b=9, q=1, e=1, q2=6, e2=0, ambig=3),
               dict(a=2, b=4, q=4, e=2, q2=24, e2=1, ambig=1),
               dict(a=1, b=6, q=0, e=1, q2=2, e2=0, ambig=6)):
        for w in (-1, 3, 40, 700):
            for Z in (-1, 0, 25):
                b = seqgen.from_lists(T, Q, sc, w, Z)
                want, _ = oracle_align(b)
                assert_same(gpu_align(b), want, b, f"boundary sc={sc} w={w} Z={Z}")


@pytest.mark.parametrize("w", [-1, 300, 751, 2000])
def test_sliding_window_short_by_long(w):
    """One short and one long sequence: the band is wider than one wave
    holds, but a single wave whose window follows the anti-diagonals' cells
    runs the pair. Short target or short query (the window moves down or
    up), related and unrelated pairs (z-drops mid-way), N bases, and a short
    side near the sliding limit of each class."""
    import paper_2403_06478_amd as ga
    rng = np.random.default_rng(9000 + max(w, 0))
    T, Q = [], []
    def seq(alphabet, k, p=None):
        return rng.choice(np.frombuffer(alphabet, dtype=np.uint8), k, p=p).tobytes()

    for k in range(36):
        s = int(rng.choice([3, 40, 150, 240, 470]))
        # unbanded: keep 2 * max_len + 1 within the 8180 diagonals the host accepts
        l = int(rng.integers(1500, 4000 if w < 0 else 6000))
        base = seq(b"ACGT", l)
        if k % 3 == 0:
            short = seq(b"ACGTN", s, p=[0.24, 0.24, 0.24, 0.24, 0.04])
        else:
            off = int(rng.integers(0, max(1, min(l - s, 60))))
            short = bytearray(base[off:off + s])
            for t in range(len(short)):
                if rng.random() < 0.08:
                    short[t] = b"ACGT"[int(rng.integers(0, 4))]
            short = bytes(short)
        if k % 2 == 0:
            T.append(short)
            Q.append(base)
        else:
            T.append(base)
            Q.append(short)
    # short sides exactly at and one past each sliding window's limit
    # (2s + 11 + K <= 64K: s <= 120 for K=4, s <= 246 for K=8, s <= 498 for
    # K=16), both ways
    for s in (120, 121, 246, 247, 498, 499):
        base = seq(b"ACGT", int(rng.integers(3000, 4000)))
        short = base[100:100 + s]
        T += [short, base]
        Q += [base, short]
    for Z in (-1, 60, 400):
        b = seqgen.from_lists(T, Q, seqgen.SCORING, w, Z)
        cls = [ga.ga_pair_class(int(n), int(m), w) for n, m in zip(b.t_len, b.q_len)]
        _say(f"sliding w={w} Z={Z}: classes {sorted(set(cls))}")
        if w < 0 or w >= 300:
            assert {5, 6} & set(cls) and 11 in cls
        want, _ = oracle_align(b)
        assert_same(gpu_align(b), want, b, f"sliding w={w} Z={Z}")


def test_bucketed_schedule_same_results():
    """The plain per-length-bucket schedule (the comparison baseline) gives
    the same results as the persistent one, and both match the oracle."""
    import torch

    import paper_2403_06478_amd as ga
    full = seqgen.make_workload("mix", n_pairs=3000)
    idx = np.nonzero(full.t_len <= 6000)[0][:1200]
    b = full.subset(idx)
    ctx = ga.Context(0)
    packed = ga.pack_batch(ctx, b)
    outs = {}
    for sched in ("bucketed", "unordered", "persistent"):
        ctx.set_schedule(sched)
        out = ga.ga_align_batch(ctx, packed, b.scoring, b.w, b.zdrop)
        torch.cuda.synchronize()
        ctx.check()
        outs[sched] = out.cpu().numpy()
        _say(f"schedule {sched}: {b.n_pairs} pairs")
    assert np.array_equal(outs["bucketed"], outs["persistent"])
    assert np.array_equal(outs["unordered"], outs["persistent"])
    want, _ = oracle_align(b)
    assert_same(outs["persistent"], want, b, "schedules")
    assert ga.load_library().ga_context_set_schedule(ctx._h, 7) == ga.GA_EINVAL
    ctx.close()


def test_serving_isolation():
    """Continuous batching: requests of the serving mix arrive over time and
    are served in many overlapping batches; every result equals the oracle's
    and the same request run alone."""
    import paper_2403_06478_amd as ga
    from paper_2403_06478_amd import serve
    b = seqgen.make_workload("serving", n_pairs=160, seed=3)
    arrivals = np.cumsum(np.random.default_rng(31).exponential(1.0 / 3000.0, size=b.n_pairs))
    # small rings (twice a batch) so requests wait for ring space and the
    # ring wraps around
    res, lat, wall, nb = serve.serve_trace(b, arrivals, slots=2, long_slots=1, max_batch_pairs=8,
                                           max_batch_bases=6000, long_batch_pairs=8,
                                           long_batch_bases=40000, ring_factor=2)
    _say(f"served {b.n_pairs} requests in {nb} batches, {wall * 1e3:.1f} ms, p99 {np.percentile(lat, 99) * 1e3:.2f} ms")
    assert nb > 3
    assert np.all(lat > 0)
    want, _ = oracle_align(b)
    assert_same(res, want, b, "served")
    for k in range(0, b.n_pairs, 7):
        alone = gpu_align(b.subset([k]))
        assert np.array_equal(alone[0], res[k]), (k, alone[0].tolist(), res[k].tolist())


def _short_by_long(rng, n_pairs, t_lo, t_hi, q_lo, q_hi, w, Z=400):
    """Long targets against short queries copied (with 5% substitutions)
    from a random place of the target."""
    acgt = np.frombuffer(b"ACGT", dtype=np.uint8)
    T, Q = [], []
    for _ in range(n_pairs):
        n = int(rng.integers(t_lo, t_hi + 1))
        m = int(rng.integers(q_lo, q_hi + 1))
        t = acgt[rng.integers(0, 4, n)]
        s0 = int(rng.integers(0, n - m + 1))
        q = t[s0:s0 + m].copy()
        sub = rng.random(m) < 0.05
        q[sub] = acgt[rng.integers(0, 4, int(sub.sum()))]
        T.append(t.tobytes())
        Q.append(q.tobytes())
    return seqgen.from_lists(T, Q, seqgen.SCORING, w, Z)


def test_every_class_same_results():
    """The result does not depend on the kernel shape: pairs forced onto each
    class that runs them (ga_context_set_classes) give the default choice's
    results, which match the oracle. Covers every class, fixed, sliding and
    multi-wave, on bands each shape holds."""
    import torch

    import paper_2403_06478_amd as ga
    rng = np.random.default_rng(41)
    scenarios = [
        ("fixed w=100", seqgen.random_pairs(rng, 40, 300, 700, err=0.05, w=100, zdrop=400), [0, 1, 2, 3, 4]),
        ("sliding K8", _short_by_long(rng, 16, 1500, 2500, 60, 240, 751), [5, 2, 3, 4]),
        ("sliding K16", _short_by_long(rng, 16, 1500, 2500, 280, 490, 751), [6, 3, 4]),
        ("w=1000", seqgen.random_pairs(rng, 10, 2200, 2600, err=0.05, w=1000, zdrop=400), [4, 7]),
        ("w=1500", seqgen.random_pairs(rng, 8, 3200, 3500, err=0.05, w=1500, zdrop=400), [7, 8]),
        ("w=2500", seqgen.random_pairs(rng, 4, 2700, 3000, err=0.05, w=2500, zdrop=400), [9]),
        ("w=3500", seqgen.random_pairs(rng, 3, 3600, 3800, err=0.05, w=3500, zdrop=400), [10]),
        ("sliding K4", _short_by_long(rng, 16, 1500, 2500, 20, 115, 751), [11, 5, 2, 3, 4]),
        ("small-K waves w=400", seqgen.random_pairs(rng, 12, 900, 1100, err=0.05, w=400, zdrop=400),
         [2, 12, 14]),
        ("small-K waves w=200", seqgen.random_pairs(rng, 16, 500, 700, err=0.05, w=200, zdrop=300), [1, 13]),
    ]
    ctx = ga.Context(0)
    for label, b, classes in scenarios:
        packed = ga.pack_batch(ctx, b)
        _say(f"classes {label}: default, {b.n_pairs} pairs")
        ref = ga.ga_align_batch(ctx, packed, b.scoring, b.w, b.zdrop)
        torch.cuda.synchronize()
        ctx.check()
        ref = ref.cpu().numpy()
        want, _ = oracle_align(b)
        assert_same(ref, want, b, label)
        for c in classes:
            idx = [p for p in range(b.n_pairs)
                   if ga.ga_pair_class_in(int(b.t_len[p]), int(b.q_len[p]), b.w, [c]) == c]
            assert len(idx) >= max(1, b.n_pairs // 2), (label, c, len(idx))
            sub = b.subset(idx)
            ctx.set_classes([c])
            _say(f"classes {label}: {ga.class_name(c)} on {len(idx)} pairs")
            got = ga.ga_align_batch(ctx, ga.pack_batch(ctx, sub), sub.scoring, sub.w, sub.zdrop)
            torch.cuda.synchronize()
            ctx.check()
            assert_same(got.cpu().numpy(), ref[idx], sub, f"{label} class {c}")
            ctx.set_classes(None)
    ctx.close()


def _prefix_then_random(rng, n_pairs, lo, hi, pre_lo, pre_hi):
    """Pairs that share a prefix of U{pre_lo..pre_hi} bases and are unrelated
    after it: the global maximum is taken early and never moves again."""
    acgt = np.frombuffer(b"ACGT", dtype=np.uint8)
    T, Q = [], []
    for _ in range(n_pairs):
        n, m = (int(x) for x in rng.integers(lo, hi + 1, 2))
        k = int(rng.integers(pre_lo, pre_hi + 1))
        t = acgt[rng.integers(0, 4, n)]
        q = acgt[rng.integers(0, 4, m)]
        q[:k] = t[:k]
        T.append(t.tobytes())
        Q.append(q.tobytes())
    return T, Q


def test_k24_narrow_triangles():
    """The 24-slot class runs its start and end triangles with 16 slots per
    lane and moves the state between the layouts: results match the oracle
    when the sweep ends in each phase, when z-drop fires in each phase, when
    the global maximum is still parked at a hand-off, on lopsided bands
    (a0 = -m), unbanded, and right above the 16-slot capacity."""
    import paper_2403_06478_amd as ga
    rng = np.random.default_rng(77)
    sc = dict(seqgen.SCORING)
    cases = []
    b = seqgen.random_pairs(rng, 60, 270, 2200, err=0.1, n_rate=0.002, w=751, zdrop=400)
    cases.append(("w=751 lengths 270..2200", b))
    b = seqgen.random_pairs(rng, 40, 400, 2500, err=0.15, related=0.6, w=751, zdrop=60)
    cases.append(("w=751 drops", b))
    T, Q = _prefix_then_random(rng, 24, 600, 1800, 100, 260)
    cases.append(("prefix then random, no z-drop", seqgen.from_lists(T, Q, sc, 751, -1)))
    cases.append(("prefix then random, Z=300", seqgen.from_lists(T, Q, sc, 751, 300)))
    cases.append(("lopsided a0=-m, drops", _short_by_long(rng, 20, 1800, 3000, 540, 760, 751)))
    acgt = np.frombuffer(b"ACGT", dtype=np.uint8)
    T, Q = [], []
    for _ in range(20):  # query = the target's first m bases, 5% substituted
        n, m = int(rng.integers(1800, 3001)), int(rng.integers(540, 761))
        t = acgt[rng.integers(0, 4, n)]
        q = t[:m].copy()
        sub = rng.random(m) < 0.05
        q[sub] = acgt[rng.integers(0, 4, int(sub.sum()))]
        T.append(t.tobytes())
        Q.append(q.tobytes())
    cases.append(("lopsided a0=-m, to the query's end", seqgen.from_lists(T, Q, sc, 751, 400)))
    b = seqgen.random_pairs(rng, 30, 520, 760, err=0.08, w=-1, zdrop=-1)
    cases.append(("unbanded n+m<1536", b))
    for w in (512, 520, 600):
        b = seqgen.random_pairs(rng, 20, 500, 1500, err=0.1, w=w, zdrop=400)
        cases.append((f"w={w}", b))
    for label, b in cases:
        cls = [ga.ga_pair_class(int(b.t_len[p]), int(b.q_len[p]), b.w) for p in range(b.n_pairs)]
        n24 = sum(c == 3 for c in cls)
        _say(f"k24 triangles: {label}: {b.n_pairs} pairs, {n24} in the 24-slot class")
        assert n24 >= b.n_pairs // 2, (label, n24)
        want, _ = oracle_align(b)
        assert_same(gpu_align(b), want, b, label)


def test_k16_narrow_triangles():
    """The 16-slot class runs its start and end triangles with 8 slots per
    lane: the same hand-offs as the 24-slot class's, on bands of 513-1024
    diagonals (short pairs inside a wide band, whose whole sweep is start
    and end triangle, long pairs in a narrow band, lopsided, unbanded,
    drops, a parked maximum at a hand-off)."""
    import paper_2403_06478_amd as ga
    rng = np.random.default_rng(78)
    sc = dict(seqgen.SCORING)
    cases = []
    cases.append(("w=751 lengths 260..510", seqgen.random_pairs(rng, 60, 260, 510, err=0.1, n_rate=0.002,
                                                                  w=751, zdrop=400)))
    cases.append(("w=751 drops", seqgen.random_pairs(rng, 40, 270, 500, err=0.15, related=0.6, w=751,
                                                      zdrop=40)))
    for w in (257, 300, 400, 511):
        cases.append((f"w={w}", seqgen.random_pairs(rng, 20, 600, 1600, err=0.1, w=w, zdrop=400)))
    T, Q = _prefix_then_random(rng, 24, 600, 1400, 60, 180)
    cases.append(("prefix then random, no z-drop", seqgen.from_lists(T, Q, sc, 400, -1)))
    cases.append(("prefix then random, Z=200", seqgen.from_lists(T, Q, sc, 400, 200)))
    acgt = np.frombuffer(b"ACGT", dtype=np.uint8)
    T, Q = [], []
    for _ in range(20):  # query = the target's first m bases, 5% substituted
        n, m = int(rng.integers(1000, 2001)), int(rng.integers(260, 381))
        t = acgt[rng.integers(0, 4, n)]
        q = t[:m].copy()
        sub = rng.random(m) < 0.05
        q[sub] = acgt[rng.integers(0, 4, int(sub.sum()))]
        T.append(t.tobytes())
        Q.append(q.tobytes())
    cases.append(("lopsided a0=-m", seqgen.from_lists(T, Q, sc, 400, 400)))
    cases.append(("unbanded n+m<1024", seqgen.random_pairs(rng, 30, 270, 500, err=0.08, w=-1, zdrop=-1)))
    for label, b in cases:
        cls = [ga.ga_pair_class(int(b.t_len[p]), int(b.q_len[p]), b.w) for p in range(b.n_pairs)]
        n16 = sum(c == 2 for c in cls)
        _say(f"k16 triangles: {label}: {b.n_pairs} pairs, {n16} in the 16-slot class")
        assert n16 >= b.n_pairs // 2, (label, n16)
        want, _ = oracle_align(b)
        assert_same(gpu_align(b), want, b, label)


def test_class_mask_errors():
    """A pair that no allowed class runs is flagged and latches GA_EDEVICE;
    the other pairs are unaffected; bad masks are rejected."""
    import torch

    import paper_2403_06478_amd as ga
    rng = np.random.default_rng(43)
    b = seqgen.random_pairs(rng, 12, 100, 900, err=0.05, w=300, zdrop=400)
    ok = np.array([ga.ga_pair_class_in(int(n), int(m), b.w, [0]) == 0 for n, m in zip(b.t_len, b.q_len)])
    assert ok.any() and not ok.all()
    ctx = ga.Context(0)
    lib = ga.load_library()
    assert lib.ga_context_set_classes(ctx._h, 0) == ga.GA_EINVAL
    assert lib.ga_context_set_classes(ctx._h, 1 << len(ga.CLASSES)) == ga.GA_EINVAL
    packed = ga.pack_batch(ctx, b)
    ctx.set_classes([0])
    out = ga.ga_align_batch(ctx, packed, b.scoring, b.w, b.zdrop)
    torch.cuda.synchronize()
    with pytest.raises(ga.GaError) as ei:
        ctx.check()
    assert ei.value.code == ga.GA_EDEVICE
    got = out.cpu().numpy()
    assert np.all(got[~ok] == np.array([0, -1, -1, 0, -1, -1, -1]))
    want, _ = oracle_align(b)
    assert_same(got[ok], want[ok], b.subset(np.nonzero(ok)[0]), "mask errors")
    ctx.set_classes(None)
    ctx.check()
    ctx.close()


def test_cli_fasta(tmp_path):
    """The FASTA front end: wrapped, mixed-case records with N and an empty
    record, aligned record by record; score.log matches the oracle."""
    import json

    from paper_2403_06478_amd import cli
    rng = np.random.default_rng(47)
    b = seqgen.random_pairs(rng, 30, 0, 700, err=0.08, n_rate=0.01, related=0.9, w=200, zdrop=100)
    T = [bytes(x if (k % 7) else x | 0x20 for k, x in enumerate(b.target(p))) for p in range(b.n_pairs)]
    Q = [b.query(p) for p in range(b.n_pairs)]
    T[3] = b""

    def write(path, seqs, tag):
        with open(path, "wb") as f:
            for k, s in enumerate(seqs):
                f.write(f">{tag}{k} record {k}\n".encode())
                for o in range(0, len(s), 60):
                    f.write(s[o:o + 60] + b"\n")

    write(tmp_path / "ref.fa", T, "r")
    write(tmp_path / "qry.fa", Q, "q")
    out = tmp_path / "out"
    _say("cli: 30 records")
    assert cli.main([str(tmp_path / "ref.fa"), str(tmp_path / "qry.fa"), "-a", "2", "-b", "4", "-q", "4",
                     "-r", "2", "-z", "100", "-w", "200", "-o", str(out)]) == 0
    rows = [line.split("\t") for line in (out / "score.log").read_text().splitlines() if not line.startswith("#")]
    assert [r[0] for r in rows] == [f"r{k} record {k}" for k in range(b.n_pairs)]
    got = np.array([[int(x) for x in r[2:]] for r in rows], dtype=np.int32)
    want, _ = oracle_align(seqgen.from_lists(T, Q, seqgen.SCORING, 200, 100))
    assert_same(got, want, None, "cli")
    meta = json.loads((out / "time.json").read_text())
    assert meta["pairs"] == b.n_pairs and meta["kernel_ms"] > 0


def test_graph_replays_match_eager():
    """A serving slot replays one captured HIP graph (packing out of the
    pinned request ring and aligning, at the slot's capacity) for batches of
    different sizes; every replay, with eager work and synchronisation
    between replays, equals the eager path on the same requests and the
    oracle. One slot's graph forks the context's streams."""
    import time

    import torch

    from paper_2403_06478_amd import serve
    rng = np.random.default_rng(53)
    sc = dict(seqgen.SCORING)
    slots = {}
    for name, graphs, lanes in (("graph", True, 1), ("forked", True, 3), ("eager", False, 1)):
        slots[name] = serve._Slot(0, serve.RequestRing(30000), 16, sc, 200, 150, graphs=graphs, lanes=lanes)
    for k, n in enumerate([16, 1, 9, 16, 5]):
        b = seqgen.random_pairs(rng, n, 0, 700, err=0.1, n_rate=0.01, related=0.8, w=200, zdrop=150)
        _say(f"graph replay {k}: {n} pairs")
        got = {}
        for name, slot in slots.items():
            reqs = [serve._Request(i, b.target(i), b.query(i), 0.0) for i in range(n)]
            assert slot.ring.admit(reqs, 16) == n
            slot.launch(reqs)
        for name, slot in slots.items():
            for _ in range(20000):
                r = slot.poll()
                if r is not None:
                    got[name] = r[1]
                    break
                time.sleep(0.0005)
            assert slot.ring.space.used == 0  # the batch's ring space is released
        assert slots["graph"].graph is not None and slots["eager"].graph is None
        assert np.array_equal(got["graph"], got["eager"]), k
        assert np.array_equal(got["forked"], got["eager"]), k
        assert np.array_equal(got["graph"], gpu_align(b)), k
        want, _ = oracle_align(b)
        assert_same(got["graph"], want, b, f"graph replay {k}")
        # unrelated eager work and a full synchronisation between replays
        x = torch.arange(1 << 20, device="cuda", dtype=torch.int32)
        assert int(x.sum().item()) == (1 << 20) * ((1 << 20) - 1) // 2
        torch.cuda.synchronize()
    for slot in slots.values():
        slot.ctx.close()


def test_offline_graph_replays():
    """One whole ga_align_batch call (planning, the fork over the context's
    four streams, every class launch, the join) captured into a HIP graph:
    each of several replays -- with unrelated eager work and a full
    synchronisation between them -- equals the eager call, which matches
    the oracle. The captured call's output is cleared before every replay."""
    import torch

    import paper_2403_06478_amd as ga
    full = seqgen.make_workload("mix", n_pairs=3000, seed=7)
    b = full.subset(np.nonzero(full.t_len <= 6000)[0][:1500])
    ctx = ga.Context(0)
    packed = ga.pack_batch(ctx, b)
    eager = ga.ga_align_batch(ctx, packed, b.scoring, b.w, b.zdrop)
    torch.cuda.synchronize()
    ctx.check()
    eager = eager.cpu().numpy()
    want, _ = oracle_align(b)
    assert_same(eager, want, b, "graph eager")
    s = torch.cuda.Stream()  # default priority; capture needs a stream of its own
    out = torch.full((b.n_pairs, 7), -9, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    lib = ga.load_library()
    bad = ctypes.c_void_p()
    assert lib.ga_graph_capture(ctx.handle, ctypes.byref(packed.struct()), ctypes.byref(ga.scoring_struct(b.scoring)),
                                b.w, b.zdrop, out.data_ptr(), None, ctypes.byref(bad)) == ga.GA_EINVAL
    g = ga.AlignGraph(ctx, packed, b.scoring, b.w, b.zdrop, out, s)
    for k in range(3):
        out.fill_(-9)
        torch.cuda.synchronize()
        _say(f"offline graph replay {k}: {b.n_pairs} pairs")
        g.launch(s)
        s.synchronize()
        ctx.check()
        assert np.array_equal(out.cpu().numpy(), eager), k
        x = torch.arange(1 << 20, device="cuda", dtype=torch.int32)
        assert int(x.sum().item()) == (1 << 20) * ((1 << 20) - 1) // 2
        torch.cuda.synchronize()
    g.close()
    ctx.close()


def test_autotune_order_and_results():
    """The autotuner measures every class; afterwards each pair takes the
    cheapest (by the measured costs) allowed class that runs it, and the
    results under the tuned order stay those of the oracle on a batch that
    spans every fixed, sliding and multi-wave class of the mixed workload."""
    import torch

    import paper_2403_06478_amd as ga
    ctx = ga.Context(0)
    cost = ctx.autotune()
    _say("autotune: " + ", ".join(f"{ga.class_name(c)}={cost[c]:.3f}" for c in range(len(cost))))
    assert len(cost) == len(ga.CLASSES) and all(np.isfinite(cost)) and min(cost) > 0
    rng = np.random.default_rng(61)
    every = range(len(ga.CLASSES))
    for _ in range(2000):
        n, m = (int(x) for x in rng.integers(1, 9000, 2))
        w = int(rng.choice([-1, 50, 300, 751, 1000, 1500, 2500, 3500]))
        holders = [c for c in every if ga.ga_pair_class_in(n, m, w, [c]) == c]
        got = ctx.pair_class(n, m, w)
        if not holders:
            assert got == -1
            continue
        assert got in holders and cost[got] == min(cost[c] for c in holders), (n, m, w, got, holders)
    full = seqgen.make_workload("mix", n_pairs=3000, seed=5)
    b = full.subset(np.nonzero(full.t_len <= 6000)[0][:1200])
    classes = sorted({ctx.pair_class(int(n), int(m), b.w) for n, m in zip(b.t_len, b.q_len)})
    _say(f"autotuned mix sample: {b.n_pairs} pairs in classes {classes}")
    packed = ga.pack_batch(ctx, b)
    out = ga.ga_align_batch(ctx, packed, b.scoring, b.w, b.zdrop)
    torch.cuda.synchronize()
    ctx.check()
    want, _ = oracle_align(b)
    assert_same(out.cpu().numpy(), want, b, "autotuned mix sample")
    ctx.close()


def test_latency_order_small_batches():
    """After autotuning, a call of few pairs plans with the classes ordered
    by measured latency (a batch that does not fill the GPU lasts as long
    as its longest sweep): results equal the throughput order's and the
    oracle's, and the host's class choice for such a call is the cheapest
    holder by the measured latencies."""
    import torch

    import paper_2403_06478_amd as ga
    ctx = ga.Context(0)
    cost = ctx.autotune()
    lat = ctx.class_latency()
    _say("latency ns/anti-diagonal: " + ", ".join(f"{ga.class_name(c)} {lat[c]:.1f}" for c in range(len(lat))))
    assert len(lat) == len(ga.CLASSES) and all(np.isfinite(lat)) and min(lat) > 0
    rng = np.random.default_rng(61)
    b = seqgen.random_pairs(rng, 300, 100, 1000, err=0.05, n_rate=0.002, related=0.9, w=500, zdrop=400)
    every = range(len(ga.CLASSES))
    for n, m in zip(b.t_len[:60], b.q_len[:60]):
        holders = [c for c in every if ga.ga_pair_class_in(int(n), int(m), b.w, [c]) == c]
        got = ctx.pair_class(int(n), int(m), b.w, b.n_pairs)
        assert got == min(holders, key=lambda c: (lat[c], holders.index(c))), (n, m, got, holders)
    packed = ga.pack_batch(ctx, b)
    small = ga.ga_align_batch(ctx, packed, b.scoring, b.w, b.zdrop)
    torch.cuda.synchronize()
    ctx.check()
    ctx.set_latency_pairs(0)  # the throughput order for every call
    big = ga.ga_align_batch(ctx, packed, b.scoring, b.w, b.zdrop)
    torch.cuda.synchronize()
    ctx.check()
    assert np.array_equal(small.cpu().numpy(), big.cpu().numpy())
    want, _ = oracle_align(b)
    assert_same(small.cpu().numpy(), want, b, "latency order")
    used = sorted({ctx.pair_class(int(n), int(m), b.w, b.n_pairs) for n, m in zip(b.t_len, b.q_len)})
    _say(f"latency order off: classes {used}")
    ctx.close()


def test_lanes_same_results():
    """Spreading the class launches over one to four streams gives the same
    results (checked against the oracle on a mixed sample)."""
    import torch

    import paper_2403_06478_amd as ga
    full = seqgen.make_workload("mix", n_pairs=3000, seed=4)
    b = full.subset(np.nonzero(full.t_len <= 6000)[0][:1500])
    ctx = ga.Context(0)
    lib = ga.load_library()
    assert lib.ga_context_set_lanes(ctx._h, 0) == ga.GA_EINVAL
    assert lib.ga_context_set_lanes(ctx._h, 5) == ga.GA_EINVAL
    packed = ga.pack_batch(ctx, b)
    outs = []
    for lanes in (1, 2, 3, 4):
        ctx.set_lanes(lanes)
        ctx.set_timing(True)
        out = ga.ga_align_batch(ctx, packed, b.scoring, b.w, b.zdrop)
        torch.cuda.synchronize()
        ctx.check()
        ms = ctx.timing()
        assert all(x >= 0 for x in ms) and sum(ms[1:]) > 0
        outs.append(out.cpu().numpy())
        _say(f"lanes {lanes}: {b.n_pairs} pairs, stages {[round(x, 3) for x in ms]}")
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    want, _ = oracle_align(b)
    assert_same(outs[-1], want, b, "lanes")
    ctx.close()


def test_native_server():
    """The native server (C++ host loop over the same slots, rings and
    graphs): a trace served through small rings gives the oracle's results,
    the same as the Python loop's; submit and poll work one by one too."""
    import time

    import paper_2403_06478_amd as ga
    from paper_2403_06478_amd import serve
    b = seqgen.make_workload("serving", n_pairs=160, seed=3)
    arrivals = np.cumsum(np.random.default_rng(31).exponential(1.0 / 3000.0, size=b.n_pairs))
    kw = dict(slots=2, long_slots=1, max_batch_pairs=8, max_batch_bases=6000, long_batch_pairs=8,
              long_batch_bases=40000, ring_factor=2)
    res, lat, wall, nb = serve.serve_trace_native(b, arrivals, **kw)
    _say(f"native: {b.n_pairs} requests in {nb} batches, {wall * 1e3:.1f} ms")
    assert nb > 3 and np.all(lat > 0)
    want, _ = oracle_align(b)
    assert_same(res, want, b, "native served")
    res_py, _, _, _ = serve.serve_trace(b, arrivals, **kw)
    assert np.array_equal(res, res_py)
    # a trace cycling over the pool (request k asks for pair k mod 160), so
    # the rings wrap many times: every request gets its pair's result
    pairs = np.arange(3 * b.n_pairs) % b.n_pairs
    arr3 = np.cumsum(np.random.default_rng(32).exponential(1.0 / 6000.0, size=pairs.shape[0]))
    res3, lat3, _, _ = serve.serve_trace_native(b, arr3, pairs=pairs, **kw)
    assert np.all(lat3 > 0)
    assert np.array_equal(res3, want[pairs])
    # one by one through submit/poll, eager steps
    srv = serve.NativeServer(b.scoring, b.w, b.zdrop, 0, graphs=False, **kw)
    lib = ga.load_library()
    for k in range(20):
        t, q = b.target(k), b.query(k)
        assert lib.ga_server_submit(srv._h, k, t, len(t), q, len(q), -1.0) == ga.GA_OK
    tags = np.zeros(64, dtype=np.int64)
    out = np.zeros((64, 7), dtype=np.int32)
    got = {}
    for _ in range(40000):
        nd = lib.ga_server_poll(srv._h, tags.ctypes.data, out.ctypes.data, None, 64)
        assert nd >= 0
        for i in range(nd):
            got[int(tags[i])] = out[i].copy()
        if len(got) == 20:
            break
        time.sleep(0.0005)
    assert lib.ga_server_pending(srv._h) == 0
    assert np.array_equal(np.array([got[k] for k in range(20)]), want[:20])
    huge = b"A" * 200000
    assert lib.ga_server_submit(srv._h, 99, huge, len(huge), b"A", 1, -1.0) == ga.GA_EUNSUPPORTED
    # a collection buffer smaller than a slot's capacity (8 pairs) is refused
    assert lib.ga_server_poll(srv._h, tags.ctypes.data, out.ctypes.data, None, 7) == ga.GA_EINVAL
    assert lib.ga_server_poll(srv._h, tags.ctypes.data, out.ctypes.data, None, 0) == ga.GA_OK
    srv.close()
    # the replay deadline, forced from the host: a timeout far below one
    # batch's run returns GA_EHIP once requests are in flight; the batch
    # itself completes normally before the server is released
    long_k = int(np.argmax(b.t_len + b.q_len))
    srv = serve.NativeServer(b.scoring, b.w, b.zdrop, 0, graphs=False, replay_timeout_s=1e-6, **kw)
    with pytest.raises(ga.GaError) as ei:
        srv.replay(b, np.zeros(4), pairs=np.full(4, long_k))
    assert ei.value.code == ga.GA_EHIP
    srv.close()
