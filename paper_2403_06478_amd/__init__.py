"""Python binding of the MI355X guided extension aligner (``libga.so``).

Argument marshalling only: every step of the alignment runs in the HIP
kernels behind the C ABI of ``include/ga.h`` (same function names). PyTorch
provides device memory and streams. There is no CPU fallback: if the HIP
library is missing or no GPU is present the calls raise.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libga.so")

GA_OK = 0
GA_EINVAL = -1
GA_ENOMEM = -2
GA_EHIP = -3
GA_EUNSUPPORTED = -4
GA_EDEVICE = -5

RESULT_FIELDS = ("max_score", "max_i", "max_j", "end_score", "end_i", "end_j", "zdropped")

# Exported symbols of libga.so, as declared in include/ga.h.
ABI_SYMBOLS = ("ga_context_create", "ga_context_destroy", "ga_context_check", "ga_strerror",
               "ga_pack_words", "ga_pack", "ga_align_batch", "ga_count_cells",
               "ga_context_set_timing", "ga_context_timing", "ga_pair_class",
               "ga_calibrate_valu", "ga_context_set_schedule", "ga_context_set_classes",
               "ga_pair_class_in", "ga_context_autotune", "ga_context_pair_class", "ga_context_set_lanes",
               "ga_host_device_pointer", "ga_server_create", "ga_server_destroy", "ga_server_submit",
               "ga_server_poll", "ga_server_pending", "ga_server_batches", "ga_server_replay",
               "ga_align_batch_noalloc", "ga_graph_capture", "ga_graph_launch", "ga_graph_destroy",
               "ga_context_class_latency", "ga_context_set_latency_pairs", "ga_context_batch_class")

GA_SCHED_PERSISTENT = 0
GA_SCHED_BUCKETED = 1
GA_SCHED_UNORDERED = 2
SCHEDULES = {"persistent": GA_SCHED_PERSISTENT, "bucketed": GA_SCHED_BUCKETED, "unordered": GA_SCHED_UNORDERED}

# Alignment kernels by class: (slots per lane K, waves per pair, sliding
# window). A fixed class holds bands of up to 64 * K * waves diagonals; a
# sliding one-wave class runs a short-by-long pair whose band is wider.
CLASSES = ((4, 1, False), (8, 1, False), (16, 1, False), (24, 1, False), (32, 1, False),
           (8, 1, True), (16, 1, True), (24, 2, False), (32, 2, False), (32, 3, False), (32, 4, False),
           (4, 1, True), (8, 2, False), (4, 2, False), (4, 4, False))
CLASS_SLOTS = tuple(k for k, _, _ in CLASSES)
def class_capacity(c: int) -> int:
    """Diagonals class c holds: 64 K on one wave; neighbouring waves of a
    multi-wave class overlap by 4 diagonals (their ghost copies)."""
    k, nw, _ = CLASSES[c]
    return 64 * k + (nw - 1) * (64 * k - 4)


MAX_DIAGONALS = class_capacity(10)


def class_name(c: int) -> str:
    k, nw, sl = CLASSES[c]
    return f"ga_dp_kernel<{k},{nw},{'sliding' if sl else 'fixed'}>"


class GaError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class Scoring(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in ("a", "b", "q", "e", "q2", "e2", "ambig")]


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("slots", ctypes.c_int32), ("long_slots", ctypes.c_int32),
        ("max_batch_pairs", ctypes.c_int32), ("long_batch_pairs", ctypes.c_int32),
        ("max_batch_bases", ctypes.c_int64), ("long_batch_bases", ctypes.c_int64),
        ("long_bases", ctypes.c_int32), ("ring_factor", ctypes.c_int32), ("graphs", ctypes.c_int32),
        ("replay_timeout_s", ctypes.c_double),
    ]


class Batch(ctypes.Structure):
    _fields_ = [
        ("n_pairs", ctypes.c_int64),
        ("t_words_dev", ctypes.c_void_p), ("t_nwords", ctypes.c_int64),
        ("q_words_dev", ctypes.c_void_p), ("q_nwords", ctypes.c_int64),
        ("t_off_dev", ctypes.c_void_p), ("q_off_dev", ctypes.c_void_p),
        ("t_len_dev", ctypes.c_void_p), ("q_len_dev", ctypes.c_void_p),
        ("t_nmask_dev", ctypes.c_void_p), ("q_nmask_dev", ctypes.c_void_p),
        ("max_len", ctypes.c_int32),
    ]


_lib = None


def load_library() -> ctypes.CDLL:
    """Load ``libga.so`` (built in-tree by ``build.build()``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    # torch ships its own HIP runtime under the same soname as the system's.
    # Loading torch first makes libga.so bind to that one runtime; loaded the
    # other way round, the process would hold two runtimes and torch would
    # find no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.ga_context_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.ga_context_create.restype = ctypes.c_int
    lib.ga_context_destroy.argtypes = [vp]
    lib.ga_context_destroy.restype = ctypes.c_int
    lib.ga_context_check.argtypes = [vp, vp]
    lib.ga_context_check.restype = ctypes.c_int
    lib.ga_strerror.argtypes = [ctypes.c_int]
    lib.ga_strerror.restype = ctypes.c_char_p
    lib.ga_pack_words.argtypes = [vp, i64]
    lib.ga_pack_words.restype = i64
    lib.ga_pack.argtypes = [vp, vp, vp, vp, i64, i64, vp, vp, vp, vp]
    lib.ga_pack.restype = ctypes.c_int
    lib.ga_align_batch.argtypes = [vp, ctypes.POINTER(Batch), ctypes.POINTER(Scoring), i32, i32, vp, vp]
    lib.ga_align_batch.restype = ctypes.c_int
    lib.ga_align_batch_noalloc.argtypes = [vp, ctypes.POINTER(Batch), ctypes.POINTER(Scoring), i32, i32, vp, vp]
    lib.ga_align_batch_noalloc.restype = ctypes.c_int
    lib.ga_context_class_latency.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int]
    lib.ga_context_class_latency.restype = ctypes.c_int
    lib.ga_context_set_latency_pairs.argtypes = [vp, i32]
    lib.ga_context_set_latency_pairs.restype = ctypes.c_int
    lib.ga_context_batch_class.argtypes = [vp, i32, i32, i32, i64]
    lib.ga_context_batch_class.restype = ctypes.c_int
    lib.ga_graph_capture.argtypes = [vp, ctypes.POINTER(Batch), ctypes.POINTER(Scoring), i32, i32, vp, vp,
                                     ctypes.POINTER(vp)]
    lib.ga_graph_capture.restype = ctypes.c_int
    lib.ga_graph_launch.argtypes = [vp, vp]
    lib.ga_graph_launch.restype = ctypes.c_int
    lib.ga_graph_destroy.argtypes = [vp]
    lib.ga_graph_destroy.restype = ctypes.c_int
    lib.ga_count_cells.argtypes = [i32, i32, i32, i32]
    lib.ga_count_cells.restype = i64
    lib.ga_context_set_timing.argtypes = [vp, ctypes.c_int]
    lib.ga_context_set_timing.restype = ctypes.c_int
    lib.ga_context_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int]
    lib.ga_context_timing.restype = ctypes.c_int
    lib.ga_calibrate_valu.argtypes = [vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.ga_calibrate_valu.restype = ctypes.c_int
    lib.ga_context_set_schedule.argtypes = [vp, ctypes.c_int]
    lib.ga_context_set_schedule.restype = ctypes.c_int
    lib.ga_pair_class.argtypes = [i32, i32, i32]
    lib.ga_pair_class.restype = ctypes.c_int
    lib.ga_pair_class_in.argtypes = [i32, i32, i32, ctypes.c_uint32]
    lib.ga_pair_class_in.restype = ctypes.c_int
    lib.ga_context_set_classes.argtypes = [vp, ctypes.c_uint32]
    lib.ga_context_set_classes.restype = ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    lib.ga_server_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(Scoring), i32, i32,
                                     ctypes.POINTER(ServerConfig)]
    lib.ga_server_create.restype = ctypes.c_int
    lib.ga_server_destroy.argtypes = [vp]
    lib.ga_server_destroy.restype = ctypes.c_int
    lib.ga_server_submit.argtypes = [vp, i64, vp, i32, vp, i32, ctypes.c_double]
    lib.ga_server_submit.restype = ctypes.c_int
    lib.ga_server_poll.argtypes = [vp, vp, vp, vp, ctypes.c_int]
    lib.ga_server_poll.restype = ctypes.c_int
    lib.ga_server_pending.argtypes = [vp]
    lib.ga_server_pending.restype = i64
    lib.ga_server_batches.argtypes = [vp]
    lib.ga_server_batches.restype = i64
    lib.ga_server_replay.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, i64, vp, vp, dp]
    lib.ga_server_replay.restype = ctypes.c_int
    lib.ga_host_device_pointer.argtypes = [vp, ctypes.POINTER(vp)]
    lib.ga_host_device_pointer.restype = ctypes.c_int
    lib.ga_context_set_lanes.argtypes = [vp, ctypes.c_int]
    lib.ga_context_set_lanes.restype = ctypes.c_int
    lib.ga_context_autotune.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int, vp]
    lib.ga_context_autotune.restype = ctypes.c_int
    lib.ga_context_pair_class.argtypes = [vp, i32, i32, i32]
    lib.ga_context_pair_class.restype = ctypes.c_int
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load_library().ga_strerror(int(code)).decode()


def _check(code: int, what: str):
    if code != GA_OK:
        raise GaError(code, what)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device available: the aligner runs only on the GPU")
    return torch


def _stream_handle(stream) -> int:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def scoring_struct(sc: dict) -> Scoring:
    return Scoring(*(int(sc[k]) for k in ("a", "b", "q", "e", "q2", "e2", "ambig")))


class Context:
    """Owns a ``ga_context_t`` (device workspace) on one HIP device."""

    def __init__(self, device: int = 0):
        lib = load_library()
        self.device = int(device)
        h = ctypes.c_void_p()
        _check(lib.ga_context_create(ctypes.byref(h), self.device), "ga_context_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def check(self, stream=None):
        _check(load_library().ga_context_check(self._h, _stream_handle(stream)), "ga_context_check")

    def set_timing(self, enable: bool):
        _check(load_library().ga_context_set_timing(self._h, 1 if enable else 0), "ga_context_set_timing")

    def timing(self):
        """Stage milliseconds of the last timed call: [prep, class 0 .. class 10]."""
        n = 1 + len(CLASSES)
        ms = (ctypes.c_float * n)()
        _check(load_library().ga_context_timing(self._h, ms, n), "ga_context_timing")
        return [float(x) for x in ms]

    def set_schedule(self, schedule: str):
        """'persistent' (default), 'unordered' (persistent without the
        longest-first order) or 'bucketed' (the plain per-length-bucket
        baseline)."""
        _check(load_library().ga_context_set_schedule(self._h, SCHEDULES[schedule]), "ga_context_set_schedule")

    def set_lanes(self, lanes: int):
        """Streams (1..4) the persistent launches of one call overlap on."""
        _check(load_library().ga_context_set_lanes(self._h, int(lanes)), "ga_context_set_lanes")

    def set_classes(self, classes=None):
        """Restrict the kernel classes later calls may use (indices into
        ``CLASSES``); None allows all."""
        mask = (1 << len(CLASSES)) - 1 if classes is None else sum(1 << int(c) for c in set(classes))
        _check(load_library().ga_context_set_classes(self._h, mask), "ga_context_set_classes")

    def autotune(self, stream=None):
        """Measure every kernel class on this device and try them cheapest
        first from now on; returns the costs (ns per pair and anti-diagonal)."""
        n = len(CLASSES)
        ns = (ctypes.c_float * n)()
        _check(load_library().ga_context_autotune(self._h, ns, n, _stream_handle(stream)), "ga_context_autotune")
        return [float(x) for x in ns]

    def pair_class(self, n: int, m: int, w: int, n_pairs: Optional[int] = None) -> int:
        """The class ga_align_batch on this context picks for the pair (in a
        call of ``n_pairs`` pairs: small calls may plan by latency)."""
        if n_pairs is None:
            return int(load_library().ga_context_pair_class(self._h, int(n), int(m), int(w)))
        return int(load_library().ga_context_batch_class(self._h, int(n), int(m), int(w), int(n_pairs)))

    def class_latency(self):
        """The autotuner's per-class latency (ns per anti-diagonal of one pair
        in a batch of 64)."""
        n = len(CLASSES)
        ns = (ctypes.c_float * n)()
        _check(load_library().ga_context_class_latency(self._h, ns, n), "ga_context_class_latency")
        return [float(x) for x in ns]

    def set_latency_pairs(self, n_pairs: int):
        """Calls of at most ``n_pairs`` pairs plan by latency (0: never)."""
        _check(load_library().ga_context_set_latency_pairs(self._h, int(n_pairs)), "ga_context_set_latency_pairs")

    def calibrate_valu(self, stream=None) -> float:
        """Measured int32 VALU lane-ops per second of this device."""
        v = ctypes.c_double(0.0)
        _check(load_library().ga_calibrate_valu(self._h, ctypes.byref(v), _stream_handle(stream)),
               "ga_calibrate_valu")
        return float(v.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().ga_context_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class PackedBatch:
    """Device-resident packed pairs (2-bit streams, N bitmaps, offsets)."""

    n_pairs: int
    t_words: "object"
    t_off: "object"
    t_len: "object"
    t_nmask: "object"
    q_words: "object"
    q_off: "object"
    q_len: "object"
    q_nmask: "object"
    max_len: int

    def struct(self) -> Batch:
        b = Batch()
        b.n_pairs = self.n_pairs
        b.t_words_dev = self.t_words.data_ptr()
        b.t_nwords = self.t_words.numel()
        b.q_words_dev = self.q_words.data_ptr()
        b.q_nwords = self.q_words.numel()
        b.t_off_dev = self.t_off.data_ptr()
        b.q_off_dev = self.q_off.data_ptr()
        b.t_len_dev = self.t_len.data_ptr()
        b.q_len_dev = self.q_len.data_ptr()
        b.t_nmask_dev = self.t_nmask.data_ptr() if self.t_nmask is not None else None
        b.q_nmask_dev = self.q_nmask.data_ptr() if self.q_nmask is not None else None
        b.max_len = self.max_len
        return b


def _upload(torch, arr, dtype, device):
    arr = np.ascontiguousarray(arr)
    if arr.size == 0:
        arr = np.zeros(1, dtype=arr.dtype)
    return torch.from_numpy(arr).to(device=device, dtype=dtype)


def ga_pack(ctx: Context, ascii_seq, off, lens, stream=None):
    """Pack one side (targets or queries) on the device: ASCII bytes ->
    (words, word offsets, N bitmap, lengths) as device tensors."""
    torch = _torch()
    lib = load_library()
    dev = torch.device("cuda", ctx.device)
    lens = np.ascontiguousarray(lens, dtype=np.int32)
    n = int(lens.shape[0])
    nwords = int(lib.ga_pack_words(lens.ctypes.data, n)) if n else 0
    d_ascii = _upload(torch, np.asarray(ascii_seq, dtype=np.uint8), torch.uint8, dev)
    d_off = _upload(torch, np.asarray(off, dtype=np.int64), torch.int64, dev)
    d_len = _upload(torch, lens, torch.int32, dev)
    words = torch.empty(max(nwords, 1), dtype=torch.int32, device=dev)
    word_off = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
    nmask = torch.empty(max((nwords + 1) // 2, 1), dtype=torch.int32, device=dev)
    _check(lib.ga_pack(ctx.handle, d_ascii.data_ptr(), d_off.data_ptr(), d_len.data_ptr(), n, nwords,
                       words.data_ptr(), word_off.data_ptr(), nmask.data_ptr(), _stream_handle(stream)),
           "ga_pack")
    return words[:max(nwords, 1)], word_off, nmask, d_len, nwords


def pack_batch(ctx: Context, batch, stream=None) -> PackedBatch:
    """Pack a ``seqgen.PairBatch`` (host ASCII) into device streams."""
    tw, to, tm, tl, tn = ga_pack(ctx, batch.t_seq, batch.t_off, batch.t_len, stream)
    qw, qo, qm, ql, qn = ga_pack(ctx, batch.q_seq, batch.q_off, batch.q_len, stream)
    max_len = int(max(batch.t_len.max(initial=0), batch.q_len.max(initial=0)))
    return PackedBatch(batch.n_pairs, tw[:max(tn, 1)], to, tl, tm, qw[:max(qn, 1)], qo, ql, qm, max_len)


def ga_align_batch(ctx: Context, packed: PackedBatch, scoring: dict, w: int, Z: int,
                   out=None, stream=None):
    """Align every pair; returns (or fills) a device int32 tensor [n_pairs, 7]."""
    torch = _torch()
    lib = load_library()
    if out is None:
        out = torch.empty((max(packed.n_pairs, 1), 7), dtype=torch.int32,
                          device=torch.device("cuda", ctx.device))
    b = packed.struct()
    sc = scoring_struct(scoring)
    _check(lib.ga_align_batch(ctx.handle, ctypes.byref(b), ctypes.byref(sc), int(w), int(Z),
                              out.data_ptr(), _stream_handle(stream)), "ga_align_batch")
    return out[:packed.n_pairs]


def ga_align_batch_noalloc(ctx: Context, packed: PackedBatch, scoring: dict, w: int, Z: int, out,
                           stream=None):
    """As ``ga_align_batch`` through the allocation-free entry point: fills
    the caller's device int32 tensor ``out`` [>= n_pairs, 7]."""
    lib = load_library()
    b = packed.struct()
    sc = scoring_struct(scoring)
    _check(lib.ga_align_batch_noalloc(ctx.handle, ctypes.byref(b), ctypes.byref(sc), int(w), int(Z),
                                      out.data_ptr(), _stream_handle(stream)), "ga_align_batch_noalloc")
    return out[:packed.n_pairs]


NOALLOC_MAX_PAIRS = 1 << 20


class AlignGraph:
    """One ga_align_batch call captured into a HIP graph (ga_graph_capture):
    ``launch(stream)`` aligns the same batch into the same output again. The
    context, the packed batch and ``out`` must outlive it."""

    def __init__(self, ctx: Context, packed: PackedBatch, scoring: dict, w: int, Z: int, out, stream):
        self._h = ctypes.c_void_p()
        b = packed.struct()
        sc = scoring_struct(scoring)
        self._keep = (ctx, packed, out)
        _check(load_library().ga_graph_capture(ctx.handle, ctypes.byref(b), ctypes.byref(sc), int(w), int(Z),
                                               out.data_ptr(), _stream_handle(stream), ctypes.byref(self._h)),
               "ga_graph_capture")

    def launch(self, stream):
        _check(load_library().ga_graph_launch(self._h, _stream_handle(stream)), "ga_graph_launch")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().ga_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ga_pair_class(n: int, m: int, w: int) -> int:
    return int(load_library().ga_pair_class(int(n), int(m), int(w)))


def host_device_pointer(host_ptr: int) -> int:
    """Device address of pinned host memory (raises if it is not pinned)."""
    dev = ctypes.c_void_p()
    _check(load_library().ga_host_device_pointer(ctypes.c_void_p(host_ptr), ctypes.byref(dev)),
           "ga_host_device_pointer")
    return int(dev.value)


def ga_pair_class_in(n: int, m: int, w: int, classes) -> int:
    """The class ``ga_align_batch`` picks for the pair among ``classes`` only."""
    mask = sum(1 << int(c) for c in set(classes))
    return int(load_library().ga_pair_class_in(int(n), int(m), int(w), mask))


def ga_count_cells(n: int, m: int, w: int, r_end: int) -> int:
    return int(load_library().ga_count_cells(int(n), int(m), int(w), int(r_end)))


def count_cells(t_len, q_len, w: int, results) -> np.ndarray:
    """Algorithmic cells per pair from the results (closed form per pair)."""
    res = np.asarray(results)
    r_end = res[:, 4].astype(np.int64) + res[:, 5].astype(np.int64)
    return np.array([ga_count_cells(int(n), int(m), w, int(r)) for n, m, r in zip(t_len, q_len, r_end)],
                    dtype=np.int64)
