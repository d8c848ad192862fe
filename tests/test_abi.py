"""CPU-side checks of the C ABI: the library loads, exports every function
include/ga.h declares, and its host-only functions and argument validation
behave as documented (no GPU compute)."""

import ctypes
import os
import re

import numpy as np

import paper_2403_06478_amd as ga
from brute import band_cells

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ga.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ga_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    lib = ga.load_library()
    names = _declared_functions()
    assert names, "no declarations found"
    assert set(names) == set(ga.ABI_SYMBOLS)
    for name in names:
        assert hasattr(lib, name), name


def test_strerror_codes():
    for code in (ga.GA_OK, ga.GA_EINVAL, ga.GA_ENOMEM, ga.GA_EHIP, ga.GA_EUNSUPPORTED, ga.GA_EDEVICE):
        assert ga.strerror(code) and ga.strerror(code) != "unknown error"
    assert ga.strerror(-99) == "unknown error"


def test_count_cells_closed_form():
    rng = np.random.default_rng(0)
    for _ in range(300):
        n, m = int(rng.integers(0, 60)), int(rng.integers(0, 60))
        w = int(rng.choice([-1, 0, 1, 2, 5, 20, 100]))
        r_end = int(rng.integers(-1, n + m))
        want = band_cells(n, m, w, r_end) if n and m else 0
        assert ga.ga_count_cells(n, m, w, r_end) == want, (n, m, w, r_end)


def test_pack_words():
    lib = ga.load_library()
    lens = np.array([0, 1, 15, 16, 17, 33], dtype=np.int32)
    assert lib.ga_pack_words(lens.ctypes.data, len(lens)) == 0 + 1 + 1 + 1 + 2 + 3
    assert lib.ga_pack_words(None, 3) == -1


def test_host_validation_without_gpu():
    lib = ga.load_library()
    b = ga.Batch()
    sc = ga.scoring_struct(dict(a=2, b=4, q=4, e=2, q2=24, e2=1, ambig=1))
    # null context / null pointers are rejected before any device work
    assert lib.ga_align_batch(None, ctypes.byref(b), ctypes.byref(sc), 10, 10, None, None) == ga.GA_EINVAL
    assert lib.ga_context_create(None, 0) == ga.GA_EINVAL
    assert lib.ga_context_destroy(None) == ga.GA_EINVAL
    assert lib.ga_context_check(None, None) == ga.GA_EINVAL
    assert lib.ga_pack(None, None, None, None, 1, 1, None, None, None, None) == ga.GA_EINVAL


def test_one_hip_runtime_in_process():
    """libga.so binds to the HIP runtime torch already loaded (they share a
    soname); a second runtime in the process would hide the GPU from torch."""
    import paper_2403_06478_amd as ga
    ga.load_library()
    with open("/proc/self/maps") as f:
        paths = {line.split()[-1] for line in f if "libamdhip64" in line}
    assert len(paths) == 1, paths


def test_pair_class_rule():
    """Host class choice: the cheapest kernel that holds the pair -- a fixed
    class when the band's diagonals fit, a sliding one-wave class when the
    shorter sequence's span does, else the multi-wave classes by band."""
    import numpy as np

    import paper_2403_06478_amd as ga
    rng = np.random.default_rng(5)
    order = [0, 11, 1, 5, 2, 6, 3, 4, 7, 8, 9, 10, 13, 12, 14]
    for _ in range(3000):
        n, m = (int(x) for x in rng.integers(0, 9000, 2))
        w = int(rng.choice([-1, 0, 1, 100, 751, 1533, 1534, 2000, 2046, 3068, 4089, 4095, 5000]))
        got = ga.ga_pair_class(n, m, w)
        if n == 0 or m == 0:
            assert got == -1
            continue
        a0, a1 = (max(-w, -m), min(w, n)) if w >= 0 else (-m, n)
        D = a1 - a0 + 1
        want = -1
        for c in order:
            k, nw, sl = ga.CLASSES[c]
            cap = ga.class_capacity(c)
            if (not sl and D <= cap) or (sl and 2 * min(n, m) + 11 + k <= cap):
                want = c
                break
        assert got == want, (n, m, w, got, want)
        if got >= 0 and not ga.CLASSES[got][2]:
            assert D <= ga.class_capacity(got)


def test_pair_class_rule_restricted():
    """Class choice among a subset of the kernels: the cheapest allowed class
    that runs the pair in the shape the full rule gives it (a sliding class
    only for a band wider than its window, W waves only for a band reaching
    the last wave). With every class allowed these extra conditions never
    bind, so the choice is the full rule's."""
    import numpy as np

    import paper_2403_06478_amd as ga
    rng = np.random.default_rng(6)
    order = [0, 11, 1, 5, 2, 6, 3, 4, 7, 8, 9, 10, 13, 12, 14]
    every = range(len(ga.CLASSES))
    for _ in range(3000):
        n, m = (int(x) for x in rng.integers(1, 9000, 2))
        w = int(rng.choice([-1, 0, 100, 300, 751, 1000, 1500, 2500, 3500, 5000]))
        assert ga.ga_pair_class_in(n, m, w, every) == ga.ga_pair_class(n, m, w)
        allowed = [c for c in every if rng.random() < 0.4] or [int(rng.integers(0, len(ga.CLASSES)))]
        a0, a1 = (max(-w, -m), min(w, n)) if w >= 0 else (-m, n)
        D = a1 - a0 + 1
        want = -1
        for c in order:
            if c not in allowed:
                continue
            k, nw, sl = ga.CLASSES[c]
            cap = ga.class_capacity(c)
            if sl:
                ok = D > cap and 2 * min(n, m) + 11 + k <= cap
            else:
                below = 64 * k + (nw - 2) * (64 * k - 4) if nw > 1 else 0  # one wave fewer
                ok = below < D <= cap
            if ok:
                want = c
                break
        assert ga.ga_pair_class_in(n, m, w, allowed) == want, (n, m, w, allowed, want)


def test_fasta_reader(tmp_path):
    """FASTA records: multi-line sequences joined, blank lines and inner
    whitespace dropped, bytes kept as written; data before a header and
    unequal record counts are errors."""
    import pytest

    from paper_2403_06478_amd import cli
    ref = tmp_path / "ref.fa"
    ref.write_bytes(b">r1 first\nACGT\nacgn\n\n>r2\n\n>r3\nAC GT\r\nTT\n")
    names, seqs = cli.read_fasta(str(ref))
    assert names == ["r1 first", "r2", "r3"]
    assert seqs == [b"ACGTacgn", b"", b"ACGTTT"]
    bad = tmp_path / "bad.fa"
    bad.write_bytes(b"ACGT\n>x\nAC\n")
    with pytest.raises(ValueError):
        cli.read_fasta(str(bad))
    qry = tmp_path / "q.fa"
    qry.write_bytes(b">q1\nACGT\n")
    with pytest.raises(ValueError):
        cli.make_batch(str(ref), str(qry), dict(a=2, b=4, q=4, e=2, q2=24, e2=1, ambig=1), 10, 10)


def test_ring_space():
    """The serving ring's allocator: live regions are contiguous, inside the
    ring and disjoint; space comes back once everything older is released;
    a full ring refuses and an empty one restarts at 0."""
    import numpy as np

    from paper_2403_06478_amd.serve import RingSpace
    rng = np.random.default_rng(8)
    for cap in (64, 1000, 4096):
        sp = RingSpace(cap)
        live = {}
        for _ in range(4000):
            if live and (rng.random() < 0.45 or len(live) > 40):
                off = list(live)[int(rng.integers(0, len(live)))] if rng.random() < 0.5 else min(live, key=lambda o: live[o][1])
                sp.release(off)
                del live[off]
            else:
                size = int(rng.integers(1, max(2, cap // 3)))
                off = sp.alloc(size)
                if off < 0:
                    assert live  # only a ring with live regions refuses
                    continue
                assert 0 <= off and off + size <= cap
                for o, (sz, _) in live.items():
                    assert off + size <= o or o + sz <= off, (off, size, o, sz)
                live[off] = (size, len(live))
            assert 0 <= sp.used <= cap
        for off in list(live):
            sp.release(off)
        assert sp.used == 0 and not sp.regions and not sp.live
        assert sp.alloc(cap) == 0  # an empty ring restarts at 0
    try:
        RingSpace(10).alloc(11)
    except ValueError:
        pass
    else:
        raise AssertionError("oversized request accepted")


def test_server_config_validation_without_gpu():
    """ga_server_create refuses a bad configuration before any device work:
    counts below 1 or above the GA_SERVER_MAX_* limits of the header, a ring
    larger than its limit, a negative replay timeout; the other entry points
    refuse a null server."""
    lib = ga.load_library()
    sc = ga.scoring_struct(dict(a=2, b=4, q=4, e=2, q2=24, e2=1, ambig=1))
    text = open(HEADER).read()
    max_slots, max_pairs = 16, 1 << 20
    assert "#define GA_SERVER_MAX_SLOTS 16" in text
    assert "#define GA_SERVER_MAX_BATCH_PAIRS (1 << 20)" in text
    assert "#define GA_SERVER_MAX_RING_BYTES ((int64_t)1 << 33)" in text

    def cfg(**kw):
        base = dict(slots=2, long_slots=1, max_batch_pairs=256, long_batch_pairs=4096, max_batch_bases=10 ** 6,
                    long_batch_bases=16 * 10 ** 6, long_bases=8000, ring_factor=4, graphs=1, replay_timeout_s=0.0)
        base.update(kw)
        return ga.ServerConfig(*(base[k] for k, _ in ga.ServerConfig._fields_))

    bad = [dict(slots=0), dict(long_slots=0), dict(slots=max_slots + 1), dict(max_batch_pairs=0),
           dict(long_batch_pairs=max_pairs + 1), dict(max_batch_pairs=max_pairs + 1), dict(ring_factor=0),
           dict(max_batch_bases=0), dict(long_batch_bases=(1 << 33) // 4 + 1), dict(long_bases=-1),
           dict(replay_timeout_s=-1.0), dict(replay_timeout_s=float("nan"))]
    for kw in bad:
        h = ctypes.c_void_p()
        c = cfg(**kw)
        assert lib.ga_server_create(ctypes.byref(h), 0, ctypes.byref(sc), 500, 400, ctypes.byref(c)) == ga.GA_EINVAL, kw
        assert not h.value
    h = ctypes.c_void_p()
    assert lib.ga_server_create(ctypes.byref(h), 0, None, 500, 400, ctypes.byref(cfg())) == ga.GA_EINVAL
    assert lib.ga_server_poll(None, None, None, None, 0) == ga.GA_EINVAL
    assert lib.ga_server_submit(None, 0, b"A", 1, b"A", 1, -1.0) == ga.GA_EINVAL
    assert lib.ga_server_destroy(None) == ga.GA_EINVAL
    assert lib.ga_server_pending(None) == -1
