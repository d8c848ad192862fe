"""Independent checkers that pin the CPU oracle (no shared code with it).

* ``brute_table``: exhaustive enumeration of every band-respecting alignment
  path from the origin (-1,-1), charging each maximal gap run its two-piece
  cost gamma(l) = min(q + l*e, q2 + l*e2). It gives H(i,j) for every lattice
  point straight from the definition of the score (Section 2.1), with no
  recurrence at all. Tiny inputs only.
* ``rowmajor_table``: the recurrences of Eq. 1-3 (two-piece form) filled in
  row-major order over the whole matrix, a different evaluation order and a
  different data layout from the oracle's anti-diagonal arrays.
* ``sweep``: the anti-diagonal maximum / z-drop rule of Eq. 4-7 applied
  literally to a full table.
* ``textbook_global``: the classic three-state affine (Gotoh) global alignment
  score, one-piece gaps, no band.
"""

from __future__ import annotations

NEG = float("-inf")


def code(c: int) -> int:
    return {ord("A"): 0, ord("C"): 1, ord("G"): 2, ord("T"): 3,
            ord("a"): 0, ord("c"): 1, ord("g"): 2, ord("t"): 3}.get(c, 4)


def subst(sc: dict, x: int, y: int) -> int:
    cx, cy = code(x), code(y)
    if cx == 4 or cy == 4:
        return -sc["ambig"]
    return sc["a"] if cx == cy else -sc["b"]


def gamma(sc: dict, l: int) -> int:
    if l == 0:
        return 0
    return min(sc["q"] + l * sc["e"], sc["q2"] + l * sc["e2"])


def usable(i: int, j: int, w: int) -> bool:
    return w < 0 or abs(i - j) <= w


def brute_table(T: bytes, Q: bytes, sc: dict, w: int) -> dict:
    """H(i,j) for every reachable lattice point by enumerating all paths."""
    n, m = len(T), len(Q)
    best = {}
    # state: i, j, score, run direction ('V', 'H' or None), run length
    stack = [(-1, -1, 0, None, 0)]
    while stack:
        i, j, s, d, l = stack.pop()
        if (i, j) not in best or s > best[(i, j)]:
            best[(i, j)] = s
        if i + 1 < n and j + 1 < m and usable(i + 1, j + 1, w):
            stack.append((i + 1, j + 1, s + subst(sc, T[i + 1], Q[j + 1]), None, 0))
        if i + 1 < n and usable(i + 1, j, w):
            nl = l + 1 if d == "V" else 1
            stack.append((i + 1, j, s - (gamma(sc, nl) - gamma(sc, nl - 1)), "V", nl))
        if j + 1 < m and usable(i, j + 1, w):
            nl = l + 1 if d == "H" else 1
            stack.append((i, j + 1, s - (gamma(sc, nl) - gamma(sc, nl - 1)), "H", nl))
    return best


def rowmajor_table(T: bytes, Q: bytes, sc: dict, w: int) -> dict:
    """H(i,j) for interior in-band cells via the recurrences, row by row."""
    n, m = len(T), len(Q)
    oe1, oe2 = sc["q"] + sc["e"], sc["q2"] + sc["e2"]
    H = {}
    E1, E2, F1, F2 = {}, {}, {}, {}

    def getH(i, j):
        if not usable(i, j, w):
            return NEG
        if i == -1 and j == -1:
            return 0
        if i == -1:
            return -gamma(sc, j + 1)
        if j == -1:
            return -gamma(sc, i + 1)
        return H.get((i, j), NEG)

    for i in range(n):
        for j in range(m):
            if not usable(i, j, w):
                continue
            e1 = max(getH(i - 1, j) - oe1, E1.get((i - 1, j), NEG) - sc["e"])
            e2 = max(getH(i - 1, j) - oe2, E2.get((i - 1, j), NEG) - sc["e2"])
            f1 = max(getH(i, j - 1) - oe1, F1.get((i, j - 1), NEG) - sc["e"])
            f2 = max(getH(i, j - 1) - oe2, F2.get((i, j - 1), NEG) - sc["e2"])
            h = max(getH(i - 1, j - 1) + subst(sc, T[i], Q[j]), e1, e2, f1, f2)
            H[(i, j)], E1[(i, j)], E2[(i, j)], F1[(i, j)], F2[(i, j)] = h, e1, e2, f1, f2
    return H


def sweep(H: dict, n: int, m: int, w: int, Z: int, e2: int):
    """Eq. 4-7 applied to a full table: returns (7-tuple, cells)."""
    G, gi, gj = 0, -1, -1
    end = (0, -1, -1)
    zd = 0
    cells = 0
    if n == 0 or m == 0:
        return (0, -1, -1, 0, -1, -1, 0), 0
    for r in range(0, n + m - 1):
        diag = [(i, r - i) for i in range(max(0, r - m + 1), min(n - 1, r) + 1)
                if usable(i, r - i, w)]
        if not diag:
            continue
        cells += len(diag)
        M = max(H[c] for c in diag)
        mi, mj = min(c for c in diag if H[c] == M)
        end = (M, mi, mj)
        if M > G:
            G, gi, gj = M, mi, mj
        elif Z >= 0 and mi > gi and mj > gj and G - M > Z + e2 * abs((mi - gi) - (mj - gj)):
            zd = 1
            break
    return (int(G), gi, gj, int(end[0]), end[1], end[2], zd), cells


def band_cells(n: int, m: int, w: int, r_end: int) -> int:
    """Closed-form count of interior in-band cells on anti-diagonals 0..r_end."""
    total = 0
    for r in range(0, r_end + 1):
        lo = max(0, r - (m - 1))
        hi = min(n - 1, r)
        if w >= 0:
            lo = max(lo, -((w - r) // 2))  # ceil((r-w)/2)
            hi = min(hi, (r + w) // 2)
        if hi >= lo:
            total += hi - lo + 1
    return total


def textbook_global(T: bytes, Q: bytes, a: int, b: int, ambig: int, alpha: int, beta: int,
                    best_prefix: bool = False):
    """Three-state affine global alignment score: a gap of length l costs
    alpha + (l-1)*beta; M ends in an aligned pair, X in a gap consuming T,
    Y in a gap consuming Q. With ``best_prefix`` also returns the best global
    score over all non-empty prefix pairs, floored at 0 (the empty pair)."""
    sc = dict(a=a, b=b, ambig=ambig)
    n, m = len(T), len(Q)
    M = [[NEG] * (m + 1) for _ in range(n + 1)]
    X = [[NEG] * (m + 1) for _ in range(n + 1)]
    Y = [[NEG] * (m + 1) for _ in range(n + 1)]
    M[0][0] = 0
    for i in range(1, n + 1):
        X[i][0] = -alpha - (i - 1) * beta
    for j in range(1, m + 1):
        Y[0][j] = -alpha - (j - 1) * beta
    for i in range(1, n + 1):
        for j in range(1, m + 1):
            s = subst(sc, T[i - 1], Q[j - 1])
            M[i][j] = s + max(M[i - 1][j - 1], X[i - 1][j - 1], Y[i - 1][j - 1])
            X[i][j] = max(M[i - 1][j] - alpha, X[i - 1][j] - beta, Y[i - 1][j] - alpha)
            Y[i][j] = max(M[i][j - 1] - alpha, Y[i][j - 1] - beta, X[i][j - 1] - alpha)
    score = int(max(M[n][m], X[n][m], Y[n][m]))
    if not best_prefix:
        return score
    best = max([0] + [max(M[i][j], X[i][j], Y[i][j])
                      for i in range(1, n + 1) for j in range(1, m + 1)])
    return score, int(best)
