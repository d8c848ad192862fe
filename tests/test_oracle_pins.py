"""Pins for the CPU oracle, against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: the expected values come from
exhaustive path enumeration, an independent row-major evaluation of the
recurrences, the textbook three-state affine global alignment, closed forms
derived by hand (tests/golden/closed_forms.txt) and invariants that any
correct implementation of Section 2.1 (Eq. 1-7) must satisfy.
"""

import os

import numpy as np
import pytest

import oracle
import seqgen
from brute import band_cells, brute_table, rowmajor_table, sweep, textbook_global

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.txt")
SC = dict(seqgen.SCORING)


def _expand(spec: str) -> bytes:
    if spec == "-":
        return b""
    if "*" in spec:
        s, k = spec.split("*")
        return s.encode() * int(k)
    return spec.encode()


def _golden_cases():
    cases = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, t, q, sc, w, z, res, cells = [x.strip() for x in line.split(";")]
            a, b, qq, e, q2, e2, amb = (int(x) for x in sc.split(","))
            cases.append(dict(name=name, T=_expand(t), Q=_expand(q),
                              sc=dict(a=a, b=b, q=qq, e=e, q2=q2, e2=e2, ambig=amb),
                              w=int(w), Z=int(z), res=tuple(int(x) for x in res.split(",")),
                              cells=cells))
    return cases


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"])
def test_closed_forms(case):
    """Hand-derived values (Section 2.1, Eq. 1-7).

    * Identical ACGT sequences of length L: every diagonal cell (k,k) scores
      a*(k+1) and no path beats the diagonal; the best odd-anti-diagonal cell
      is one gap off it at a*(k+1) - gamma(1), so G - M = gamma(1) = 6 against
      a threshold Z + e2*1, and nothing drops when 6 <= Z + e2.
    * T = A^n, Q = C^n, one-piece gaps (a,b,q,e) = (2,4,4,2), Z = 400: even
      r = 2k has its maximum -(2r+4) on the diagonal (k,k) (|delta| = 0), every
      off-diagonal cell of r costs -(2r+8); odd r = 2k+1 has the value -(2r+8)
      at every cell, because stepping one diagonal further out trades a
      mismatch (-4) for two gap extensions (-4). With smallest-i ties the odd
      maximum sits at the lowest in-band i: |delta| = 1 when w is 1 or 2 (so
      the test fires at r = 199: 406 > 400 + 2), |delta| >= 3 when w >= 3
      (406 > 406 fails, the first firing is r = 200: 404 > 400). With w = 0 the
      odd anti-diagonals are empty.
    * Same pair, two-piece gaps, w = 500: up to r = 500 the maximum is the
      edge cell (0,r), -(28+r), with |delta| = r, so G - M never exceeds
      400 + r. Past the band edge every in-band cell with i, j >= 19 is
      reached by one vertical and one horizontal long-piece run,
      -(24+i+1) - (24+j+1) = -(50+r), and diagonal steps only lose; the test
      50 + r > 400 + |delta| with |delta| = 499 (odd r, edge cell
      (ceil((r-500)/2), ...)) first holds at r = 851: M = -901 at (176, 675).
      This case also fixes the slope of the z-drop rule to e2: with e = 2 the
      threshold at r = 851 would be 1398.
    * Strictness of i' < i and j' < j (Eq. 5), T = G^4 C^6, Q = G^4 with the
      benchmark scoring (gamma(l) = 4 + 2l for l <= 20), Z = 5, a band wider
      than both: even r = 2k <= 6 has the unique maximum 2(k+1) on (k,k), so
      G = 8 at (3,3) after r = 6. Odd r = 2k+1 <= 5 ties at 2(k+1) - gamma(1)
      on (k,k+1) and (k+1,k); the smallest i is (k,k+1), with
      G - M = 6 = Z + e2*1, so nothing drops there under either reading.
      The query ends at j = 3: for r = 6 + l the cells are (r-j, j), j <= 3,
      and the best is the vertical gap (3+l, 3) at 8 - gamma(l) (matching
      fewer G or placing C against G only costs more), which lies in G's
      column: mi > gi but mj = gj, so the strict rule never tests it and the
      sweep ends on the last anti-diagonal r = 12 at (9,3), 8 - gamma(6) = -8,
      after all 40 cells. A non-strict rule would test it: at r = 8,
      G - M = gamma(2) = 8 > Z + e2*2 = 7, a drop at (5,3). Swapping T and Q
      puts the same maxima in G's row (mi = gi) and pins i' < i.
    """
    res, cells = oracle.align(case["T"], case["Q"], case["sc"], case["w"], case["Z"])
    assert res == case["res"]
    if case["cells"] == "band":
        want = band_cells(len(case["T"]), len(case["Q"]), case["w"], res[4] + res[5])
    else:
        want = int(case["cells"])
    assert cells == want


def _rand_scoring(rng):
    q = int(rng.integers(0, 6))
    e = int(rng.integers(1, 4))
    return dict(a=int(rng.integers(1, 5)), b=int(rng.integers(1, 7)), q=q, e=e,
                q2=q + int(rng.integers(0, 13)), e2=int(rng.integers(0, e + 1)),
                ambig=int(rng.integers(0, 4)))


def _rand_seq(rng, n, n_rate=0.15):
    s = rng.choice(np.frombuffer(b"ACGT", dtype=np.uint8), size=n)
    s[rng.random(n) < n_rate] = ord("N")
    return s.tobytes()


def test_brute_force_tiny():
    """Every H from exhaustive path enumeration, then the Eq. 4-7 sweep, on
    random tiny pairs with random two-piece scorings, N bases, bands and
    z-drop thresholds; also the recurrences against the enumeration."""
    rng = np.random.default_rng(20240306)
    n_cases = 0
    n_dropped = 0
    for _ in range(360):
        n, m = int(rng.integers(0, 7)), int(rng.integers(0, 7))
        T, Q = _rand_seq(rng, n), _rand_seq(rng, m)
        if rng.random() < 0.5:  # related pairs make long alignments likely
            Q = T[:m] if m <= n else T + _rand_seq(rng, m - n)
        sc = _rand_scoring(rng)
        w = int(rng.choice([-1, 0, 1, 2, 3]))
        Z = int(rng.choice([-1, 0, 1, 3, 6]))
        table = brute_table(T, Q, sc, w)
        rm = rowmajor_table(T, Q, sc, w)
        for (i, j), h in rm.items():
            assert table[(i, j)] == h, (T, Q, sc, w, i, j)
        interior = {k: v for k, v in table.items() if k[0] >= 0 and k[1] >= 0}
        want, want_cells = sweep(interior, n, m, w, Z, sc["e2"])
        got, got_cells = oracle.align(T, Q, sc, w, Z)
        assert got == want, (T, Q, sc, w, Z)
        assert got_cells == want_cells
        n_cases += 1
        n_dropped += got[6]
    assert n_cases == 360 and n_dropped > 40


def test_rowmajor_moderate():
    """Row-major evaluation of the recurrences plus the literal sweep against
    the oracle on moderate random pairs (related and unrelated, with N)."""
    rng = np.random.default_rng(7)
    for k in range(40):
        b = seqgen.random_pairs(rng, 1, 20, 90, err=float(rng.choice([0.05, 0.2, 0.5])),
                                n_rate=0.03, related=0.7)
        T, Q = b.target(0), b.query(0)
        sc = _rand_scoring(rng) if k % 2 else SC
        w = int(rng.choice([-1, 0, 1, 5, 17, 40]))
        Z = int(rng.choice([-1, 0, 5, 20, 60]))
        want, want_cells = sweep(rowmajor_table(T, Q, sc, w), len(T), len(Q), w, Z, sc["e2"])
        got, got_cells = oracle.align(T, Q, sc, w, Z)
        assert got == want and got_cells == want_cells, (k, sc, w, Z)


def test_textbook_global_gotoh():
    """Unbanded, no z-drop, one-piece gaps: end_score is the textbook
    three-state affine global alignment score of the whole pair, and
    max_score is the best global score over all prefix pairs (or 0)."""
    rng = np.random.default_rng(11)
    for k in range(30):
        b = seqgen.random_pairs(rng, 1, 1, 70, err=0.15, n_rate=0.05, related=0.6)
        T, Q = b.target(0), b.query(0)
        a, bb, q, e, amb = (int(rng.integers(1, 4)), int(rng.integers(1, 6)),
                            int(rng.integers(0, 6)), int(rng.integers(1, 4)), int(rng.integers(0, 3)))
        sc = dict(a=a, b=bb, q=q, e=e, q2=q, e2=e, ambig=amb)
        got, _ = oracle.align(T, Q, sc, -1, -1)
        score, best = textbook_global(T, Q, a, bb, amb, q + e, e, best_prefix=True)
        assert got[3] == score
        assert (got[4], got[5]) == (len(T) - 1, len(Q) - 1)
        assert got[0] == best


def _batch_results(b, **kw):
    out, cells = oracle.align_batch(b, nthreads=4, **kw)
    return out, cells


def test_z_monotonicity():
    """DP values do not depend on Z: a smaller threshold stops no later, sees
    no larger maximum, and drops whenever a larger one does."""
    rng = np.random.default_rng(3)
    b = seqgen.random_pairs(rng, 120, 50, 400, err=0.12, n_rate=0.002, related=0.6, w=60)
    prev = None
    for Z in (0, 10, 40, 100, 400, -1):
        out, _ = _batch_results(b, Z=Z)
        if prev is not None:
            r_prev, r_cur = prev[:, 4] + prev[:, 5], out[:, 4] + out[:, 5]
            assert np.all(r_prev <= r_cur)
            assert np.all(prev[:, 0] <= out[:, 0])
            assert np.all(prev[:, 6] >= out[:, 6])
        prev = out
    assert prev[:, 6].sum() == 0  # Z < 0 never drops


def test_band_monotonicity():
    """Without z-drop every H and so the maximum is non-decreasing in w."""
    rng = np.random.default_rng(4)
    b = seqgen.random_pairs(rng, 80, 30, 300, err=0.2, n_rate=0.01, related=0.5)
    prev = None
    for w in (0, 1, 3, 10, 40, 200, -1):
        out, _ = _batch_results(b, w=w, Z=-1)
        if prev is not None:
            assert np.all(prev[:, 0] <= out[:, 0])
        prev = out
    # cell-level: the table of a narrower band is dominated by the wider one
    for p in range(5):
        T, Q = b.target(p)[:60], b.query(p)[:60]
        narrow, wide = rowmajor_table(T, Q, SC, 4), rowmajor_table(T, Q, SC, 9)
        assert all(h <= wide[k] for k, h in narrow.items())


def test_suffix_invariance_after_drop():
    """After a drop at anti-diagonal r_end, no base beyond index r_end of
    either sequence can matter."""
    rng = np.random.default_rng(5)
    b = seqgen.random_pairs(rng, 150, 100, 600, err=0.1, related=0.3, w=100, zdrop=50)
    out, _ = _batch_results(b)
    dropped = np.nonzero(out[:, 6])[0]
    assert len(dropped) > 30
    for p in dropped[:40]:
        r_end = int(out[p, 4] + out[p, 5])
        T, Q = bytearray(b.target(int(p))), bytearray(b.query(int(p)))
        for s in (T, Q):
            for k in range(r_end + 1, len(s)):
                s[k] = ord("ACGTN"[(s[k] + k) % 5])
        got, _ = oracle.align(bytes(T), bytes(Q), b.scoring, b.w, b.zdrop)
        assert got == tuple(out[p])


def test_score_scaling():
    """Multiplying every score parameter and Z by k scales the scores by k and
    leaves positions and the drop flag unchanged."""
    rng = np.random.default_rng(6)
    b = seqgen.random_pairs(rng, 100, 40, 300, err=0.15, n_rate=0.01, related=0.6, w=50, zdrop=30)
    base, _ = _batch_results(b)
    for k in (2, 3, 7):
        sc = {key: v * k for key, v in b.scoring.items()}
        out, _ = _batch_results(b, sc=sc, Z=b.zdrop * k)
        assert np.array_equal(out[:, [0, 3]], base[:, [0, 3]] * k)
        assert np.array_equal(out[:, [1, 2, 4, 5, 6]], base[:, [1, 2, 4, 5, 6]])


def test_symmetry_without_zdrop():
    """With Z disabled, swapping target and query leaves both scores
    unchanged (the band and the recurrences are symmetric in i and j)."""
    rng = np.random.default_rng(8)
    b = seqgen.random_pairs(rng, 100, 20, 300, err=0.2, n_rate=0.01, related=0.6)
    swapped = seqgen.from_lists([b.query(p) for p in range(b.n_pairs)],
                                [b.target(p) for p in range(b.n_pairs)])
    for w in (-1, 0, 7, 60):
        x, _ = _batch_results(b, w=w, Z=-1)
        y, _ = _batch_results(swapped, w=w, Z=-1, sc=b.scoring)
        assert np.array_equal(x[:, [0, 3]], y[:, [0, 3]])


def test_cells_formula():
    """The oracle's cell counter equals the closed-form band count up to the
    termination anti-diagonal."""
    rng = np.random.default_rng(9)
    b = seqgen.random_pairs(rng, 60, 1, 500, err=0.1, related=0.5, w=37, zdrop=40)
    out, cells = _batch_results(b)
    for p in range(b.n_pairs):
        n, m = int(b.t_len[p]), int(b.q_len[p])
        r_end = int(out[p, 4] + out[p, 5]) if n and m else -1
        assert cells[p] == band_cells(n, m, b.w, r_end)


def test_long_gap_does_not_drop():
    """Z-drop exists so that a single long indel does not end the alignment
    (Section 7). Across a 300-base insertion the gap cell costs 24 + t, which
    passes Z = 200 at t = 177, but it sits |delta| = t off the maximum's
    diagonal, so the threshold Z + e2*t is never crossed; the mismatching
    near-diagonal cells lose about 1.25 per anti-diagonal and are overtaken
    by the gap cell before they fall 200 below the maximum."""
    rng = np.random.default_rng(10)
    x = _rand_seq(rng, 400, 0.0)
    y = _rand_seq(rng, 400, 0.0)
    ins = _rand_seq(rng, 300, 0.0)
    T, Q = x + y, x + ins + y
    res, _ = oracle.align(T, Q, SC, 751, 200)
    assert res[6] == 0
    assert (res[4], res[5]) == (len(T) - 1, len(Q) - 1)
    assert res[3] == res[0] == 2 * 800 - (24 + 300)


def test_batch_matches_single():
    b = seqgen.make_workload("uniform", n_pairs=40)
    out, cells = _batch_results(b)
    for p in range(b.n_pairs):
        r, c = oracle.align(b.target(p), b.query(p), b.scoring, b.w, b.zdrop)
        assert r == tuple(out[p]) and c == cells[p]
