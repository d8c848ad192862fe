"""Continuous-batching serving loop over the C ABI.

Requests (one target/query pair each) arrive over time. Each lane of the
server (short requests, long requests) keeps a request ring in pinned,
host-coherent memory that the GPU reads in place: requests are admitted
when their bytes fit in the ring (admission by memory footprint), in groups
of at most a batch, each group written once; until then they wait in the
lane's host FIFO. A few execution slots per lane each own a context (its
own device workspace) and a HIP stream. Whenever a slot is free, the
admitted requests waiting at that moment form its next batch, up to a pair
count and a number of bases: the slot writes their ring offsets and
lengths into its pinned tables and replays one captured HIP graph that
packs both sides straight out of the ring and aligns them, the kernels
reading the tables and writing the results in pinned memory in place; no
bytes are copied per batch. Slots run concurrently, so requests
that arrive while other batches are on the GPU are admitted and batched as
soon as memory and a slot free up, and their work overlaps on the device
with the batches already running. A request's latency runs from its
arrival to the moment the host sees its batch complete; its ring space is
released once every request of its group is done.

Every step of the alignment runs in the HIP library; this module only
schedules batches and places bytes.

``python -m paper_2403_06478_amd.serve`` runs the serving benchmark: the
request mix of the ``seqgen`` workload ``serving`` with Poisson arrivals at given
fractions of the offline capacity, one JSON line per rate.
"""

from __future__ import annotations

import argparse
import collections
import ctypes
import dataclasses
import json
import sys
import time
from typing import List, Optional

import numpy as np

from . import (Batch, Context, ServerConfig, _check, _stream_handle, _torch, count_cells, ga_align_batch,
               host_device_pointer, load_library, pack_batch, scoring_struct)


@dataclasses.dataclass
class _Request:
    rid: int
    target: bytes
    query: bytes
    t_arrival: float
    off: int = -1  # ring offset of the target (the query follows it); -1 until admitted
    region: int = -1  # the ring region holding it (shared by the requests admitted together)


def _pad16(n: int) -> int:
    return (n + 15) & ~15


_ZPAD = [bytes(k) for k in range(16)]  # zero padding to the next 16-byte boundary


class RingSpace:
    """Space of a ring of `capacity` bytes handed out contiguously in
    arrival order (a request that does not fit before the end starts again
    at 0, the skipped end counting as used) and released in any order; the
    oldest released regions are reclaimed as soon as everything older is
    released too. Bookkeeping only (host side)."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self.head = 0  # next free byte
        self.used = 0  # bytes between the oldest live region and head, skipped ends included
        self.regions = collections.deque()  # [offset, size, released] in allocation order
        self.live = {}  # offset -> its region, while in use

    def alloc(self, size: int) -> int:
        """Offset of `size` contiguous bytes, or -1 if they do not fit now."""
        size = max(int(size), 1)
        if size > self.capacity:
            raise ValueError(f"{size} bytes exceed the ring ({self.capacity} bytes)")
        if self.used == 0:
            self.head = 0
        tail = (self.head - self.used) % self.capacity  # the oldest live byte
        if self.used < self.capacity and self.head >= tail:
            if self.capacity - self.head >= size:  # room before the end
                off = self.head
            elif tail >= size:  # wrap: skip the end
                skipped = self.capacity - self.head
                self.regions.append([self.head, skipped, True])
                self.used += skipped
                off = 0
            else:
                return -1
        elif self.used < self.capacity and tail - self.head >= size:  # the gap between head and tail
            off = self.head
        else:
            return -1
        reg = [off, size, False]
        self.regions.append(reg)
        self.live[off] = reg
        self.head = (off + size) % self.capacity
        self.used += size
        return off

    def release(self, off: int):
        self.live.pop(off)[2] = True
        while self.regions and self.regions[0][2]:
            self.used -= self.regions.popleft()[1]


class RequestRing:
    """The request queue of a lane: request bytes in pinned, host-coherent
    memory that the packing kernel reads in place (no copy to device memory:
    each byte crosses the bus once, when its batch is packed), laid out by a
    RingSpace. Requests are admitted in groups of at most a batch, each
    group written once into its own region, which is released when all of
    its requests are done."""

    def __init__(self, capacity: int):
        torch = _torch()
        self.space = RingSpace(_pad16(capacity))
        self.capacity = self.space.capacity
        self.buf = torch.zeros(self.capacity, dtype=torch.uint8, pin_memory=True)
        self.view = self.buf.numpy()
        # the address kernels use for the pinned buffer
        self.ptr = host_device_pointer(self.buf.data_ptr())
        self.refs = {}  # region offset -> requests in it not yet released

    def release(self, req: _Request):
        """The request is done: its region goes back once all of its
        requests are."""
        left = self.refs[req.region] - 1
        if left:
            self.refs[req.region] = left
        else:
            del self.refs[req.region]
            self.space.release(req.region)

    def admit(self, reqs, max_group: int) -> int:
        """Place the longest prefix of `reqs` (at most max_group requests)
        that fits now in one region, each request's target then its query,
        each starting on a 16-byte boundary (the packer then reads whole
        words of bases in one transaction); returns how many were placed."""
        sizes = [((len(r.target) + 15) & ~15) + ((len(r.query) + 15) & ~15) for r in reqs[:max_group]]
        k = len(sizes)
        total = sum(sizes)
        free = self.capacity - self.space.used
        while k and total > free:  # a prefix that may fit
            k -= 1
            total -= sizes[k]
        off = -1
        while k:
            off = self.space.alloc(total)
            if off >= 0:
                break
            k //= 2
            total = sum(sizes[:k])
        if k == 0:
            return 0
        if total:
            parts = []
            for r in reqs[:k]:
                parts += (r.target, _ZPAD[-len(r.target) & 15], r.query, _ZPAD[-len(r.query) & 15])
            self.view[off:off + total] = np.frombuffer(b"".join(parts), dtype=np.uint8)
        pos = off
        for r, sz in zip(reqs[:k], sizes):
            r.off, r.region = pos, off
            pos += sz
        self.refs[off] = k
        return k


class _Slot:
    """One execution slot of a lane: a context (own device workspace, one
    stream for all its launches), a HIP stream, pinned tables of ring
    offsets and lengths and a pinned result table, all sized once for the
    slot's largest batch. With ``graphs`` the device steps of a batch
    (packing both sides out of the ring and the alignment) are one captured
    HIP graph replayed per batch: every batch is presented at the slot's
    capacity (unused pair entries are empty pairs, which the planner
    finishes at once; the packed streams are declared at their full
    capacity), so one graph serves batches of any size."""

    def __init__(self, device: int, ring: RequestRing, max_pairs: int, scoring: dict, w: int, Z: int,
                 graphs: bool = True, lanes: int = 1):
        torch = _torch()
        self.lib = load_library()
        self.ctx = Context(device)
        # one stream per slot by default: the slots already overlap, and more
        # streams than the GPU's hardware queues would serialise unrelated
        # batches
        self.ctx.set_lanes(lanes)
        self.stream = torch.cuda.Stream(device=device)  # default priority
        self.ring = ring
        self.scoring, self.w, self.Z = dict(scoring), int(w), int(Z)
        self.P = P = int(max(max_pairs, 1))
        # words of one side: at most sum of ceil(len / 16) over the batch
        self.W = W = ring.capacity // 16 + P + 1
        self.max_len = min(ring.capacity, 1 << 20)  # the bound the captured call declares
        dev = torch.device("cuda", device)
        pin = dict(pin_memory=True)
        self.h_off = [torch.zeros(P, dtype=torch.int64, **pin) for _ in range(2)]
        self.h_len = [torch.zeros(P, dtype=torch.int32, **pin) for _ in range(2)]
        self.h_out = torch.zeros((P, 7), dtype=torch.int32, **pin)
        # addresses the kernels use for the pinned tables
        self.p_off = [host_device_pointer(t.data_ptr()) for t in self.h_off]
        self.p_len = [host_device_pointer(t.data_ptr()) for t in self.h_len]
        self.p_out = host_device_pointer(self.h_out.data_ptr())
        self.d_words = [torch.zeros(W, dtype=torch.int32, device=dev) for _ in range(2)]
        self.d_woff = [torch.zeros(P, dtype=torch.int64, device=dev) for _ in range(2)]
        self.d_nmask = [torch.zeros((W + 1) // 2, dtype=torch.int32, device=dev) for _ in range(2)]
        torch.cuda.synchronize(device)
        # one run on empty pairs sizes the context's workspace for the capacity
        with torch.cuda.stream(self.stream):
            self._device_steps(_stream_handle(self.stream))
        self.stream.synchronize()
        _check(self.lib.ga_context_check(self.ctx.handle, _stream_handle(self.stream)), "ga_context_check")
        self.graph = None
        if graphs:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=self.stream):
                self._device_steps(_stream_handle(torch.cuda.current_stream()))
            self.graph = g
        self.reqs: Optional[List[_Request]] = None
        self.event = None

    def _device_steps(self, st: int):
        """Pack both sides out of the ring and align, at the slot's
        capacity, all enqueued on stream st (nothing is copied)."""
        for side in range(2):
            _check(self.lib.ga_pack(self.ctx.handle, self.ring.ptr, self.p_off[side],
                                    self.p_len[side], self.P, self.W, self.d_words[side].data_ptr(),
                                    self.d_woff[side].data_ptr(), self.d_nmask[side].data_ptr(), st), "ga_pack")
        bt = Batch()
        bt.n_pairs = self.P
        bt.t_words_dev, bt.t_nwords = self.d_words[0].data_ptr(), self.W
        bt.q_words_dev, bt.q_nwords = self.d_words[1].data_ptr(), self.W
        bt.t_off_dev, bt.q_off_dev = self.d_woff[0].data_ptr(), self.d_woff[1].data_ptr()
        bt.t_len_dev, bt.q_len_dev = self.p_len[0], self.p_len[1]
        bt.t_nmask_dev, bt.q_nmask_dev = self.d_nmask[0].data_ptr(), self.d_nmask[1].data_ptr()
        bt.max_len = self.max_len
        sc = scoring_struct(self.scoring)
        _check(self.lib.ga_align_batch(self.ctx.handle, ctypes.byref(bt), ctypes.byref(sc), self.w, self.Z,
                                       self.p_out, st), "ga_align_batch")

    @property
    def busy(self) -> bool:
        return self.reqs is not None

    def launch(self, reqs: List[_Request]):
        """Start a batch of admitted requests (at most the slot's pairs)."""
        torch = _torch()
        n = len(reqs)
        if n > self.P:
            raise ValueError("batch larger than the slot")
        t_off, q_off = self.h_off[0].numpy(), self.h_off[1].numpy()
        t_len, q_len = self.h_len[0].numpy(), self.h_len[1].numpy()
        offs = np.fromiter((r.off for r in reqs), dtype=np.int64, count=n)
        nt = np.fromiter((len(r.target) for r in reqs), dtype=np.int32, count=n)
        t_off[:n], t_len[:n] = offs, nt
        q_off[:n] = offs + ((nt.astype(np.int64) + 15) & ~15)
        q_len[:n] = np.fromiter((len(r.query) for r in reqs), dtype=np.int32, count=n)
        t_off[n:], t_len[n:], q_off[n:], q_len[n:] = 0, 0, 0, 0
        with torch.cuda.stream(self.stream):
            if self.graph is not None:
                self.graph.replay()
            else:
                self._device_steps(_stream_handle(self.stream))
            self.event = torch.cuda.Event()
            self.event.record(self.stream)
        self.reqs = reqs

    def poll(self):
        """(requests, results) once the batch has completed, else None; the
        requests' ring space is released then."""
        if self.reqs is None or not self.event.query():
            return None
        _check(self.lib.ga_context_check(self.ctx.handle, _stream_handle(self.stream)), "ga_context_check")
        reqs = self.reqs
        res = self.h_out.numpy()[:len(reqs)].copy()
        for r in reqs:
            self.ring.release(r)
        self.reqs = self.event = None
        return reqs, res


class Server:
    """Continuous batching over concurrent device batches, in two lanes.

    A request whose bases (target + query) exceed ``long_bases`` goes to the
    long lane, every other request to the short lane, so short requests never
    wait behind a long pair's sweep. Each lane has its own request ring, FIFO
    and slots (``slots`` short, ``long_slots`` long). A short batch holds up
    to ``max_batch_pairs`` pairs and ``max_batch_bases`` bases; a long batch
    up to ``long_batch_pairs`` pairs and ``long_batch_bases`` bases (a long
    pair runs on one workgroup for the whole of its sweep, so a long batch
    should take every long request waiting). A request larger than its
    lane's batch limit still forms a batch of its own. The rings hold
    ``ring_factor`` times a lane's batch limit; a request larger than its
    ring is refused.

    HIP spreads streams over a few hardware queues (four by default) and the
    work of streams that share a queue runs in order, so a short batch would
    wait behind a long sweep; the defaults keep the slot streams at three
    and the server adds no other stream (the rings are read in place)."""

    def __init__(self, scoring: dict, w: int, Z: int, device: int = 0, slots: int = 2,
                 long_slots: int = 1, max_batch_pairs: int = 256, max_batch_bases: int = 1_000_000,
                 long_bases: int = 8000, long_batch_pairs: int = 4096, long_batch_bases: int = 16_000_000,
                 graphs: bool = True, ring_factor: int = 4):
        self.scoring, self.w, self.Z = dict(scoring), int(w), int(Z)
        self.pairs = [int(max_batch_pairs), int(long_batch_pairs)]
        self.limits = [int(max_batch_bases), int(long_batch_bases)]
        self.rings = [RequestRing(ring_factor * lim) for lim in self.limits]
        self.lanes = [[_Slot(device, self.rings[k], self.pairs[k], scoring, w, Z, graphs) for _ in range(n)]
                      for k, n in enumerate((slots, long_slots))]
        self.long_bases = int(long_bases)
        self.waiting = [collections.deque(), collections.deque()]   # not yet in the ring
        self.admitted = [collections.deque(), collections.deque()]  # in the ring, not yet batched
        self.batches = 0

    def submit(self, rid: int, target: bytes, query: bytes, t_arrival: Optional[float] = None):
        lane = 1 if len(target) + len(query) > self.long_bases else 0
        ring = self.rings[lane]
        if (_pad16(len(target)) + _pad16(len(query)) > ring.capacity
                or max(len(target), len(query)) > self.lanes[lane][0].max_len):
            raise ValueError(f"request {rid} is larger than its lane's ring")
        self.waiting[lane].append(_Request(rid, target, query,
                                           time.perf_counter() if t_arrival is None else t_arrival))

    @staticmethod
    def _take_batch(q, max_pairs: int, limit: int) -> List[_Request]:
        reqs, bases = [], 0
        while q and len(reqs) < max_pairs:
            r = q[0]
            size = len(r.target) + len(r.query)
            if reqs and bases + size > limit:
                break
            reqs.append(q.popleft())
            bases += size
        return reqs

    def step(self):
        """Collect finished batches (releasing their ring space), admit
        waiting requests into the rings, then start batches on free slots.
        Returns [(rid, result row, t_done)] for the requests that finished."""
        done = []
        for lane in self.lanes:
            for slot in lane:
                got = slot.poll()
                if got is not None:
                    t = time.perf_counter()
                    reqs, res = got
                    done.extend((r.rid, res[k], t) for k, r in enumerate(reqs))
        for ring, wq, aq, P in zip(self.rings, self.waiting, self.admitted, self.pairs):
            while wq:
                k = ring.admit([wq[i] for i in range(min(len(wq), P))], P)
                if not k:
                    break
                for _ in range(k):
                    aq.append(wq.popleft())
        for lane, aq, P, limit in zip(self.lanes, self.admitted, self.pairs, self.limits):
            for slot in lane:
                if not aq:
                    break
                if not slot.busy:
                    slot.launch(self._take_batch(aq, P, limit))
                    self.batches += 1
        return done

    @property
    def idle(self) -> bool:
        return (not any(self.waiting) and not any(self.admitted)
                and not any(s.busy for lane in self.lanes for s in lane))

    def close(self):
        for lane in self.lanes:
            for s in lane:
                s.ctx.close()


class NativeServer:
    """The native server (``ga_server_*`` in the library): the same lanes,
    rings, slots and graphs as ``Server``, driven by a C++ host loop."""

    def __init__(self, scoring: dict, w: int, Z: int, device: int = 0, slots: int = 2, long_slots: int = 1,
                 max_batch_pairs: int = 256, max_batch_bases: int = 1_000_000, long_bases: int = 8000,
                 long_batch_pairs: int = 4096, long_batch_bases: int = 16_000_000, graphs: bool = True,
                 ring_factor: int = 4, replay_timeout_s: float = 0.0):
        _torch()  # the HIP runtime torch uses, and a device
        self.lib = load_library()
        cfg = ServerConfig(int(slots), int(long_slots), int(max_batch_pairs), int(long_batch_pairs),
                           int(max_batch_bases), int(long_batch_bases), int(long_bases), int(ring_factor),
                           1 if graphs else 0, float(replay_timeout_s))
        sc = scoring_struct(scoring)
        h = ctypes.c_void_p()
        _check(self.lib.ga_server_create(ctypes.byref(h), int(device), ctypes.byref(sc), int(w), int(Z),
                                         ctypes.byref(cfg)), "ga_server_create")
        self._h = h

    def replay(self, batch, arrivals: np.ndarray, pairs=None):
        """Serve requests arriving at ``arrivals`` (seconds after the start);
        request k is pair ``pairs[k]`` of ``batch`` (pair k without
        ``pairs``): (results [n, 7], latencies in seconds, wall seconds)."""
        arr = np.ascontiguousarray(arrivals, dtype=np.float64)
        n = int(arr.shape[0])
        sel = np.arange(batch.n_pairs) if pairs is None else np.asarray(pairs, dtype=np.int64)
        if sel.shape[0] != n:
            raise ValueError("one arrival time per request")
        res = np.zeros((n, 7), dtype=np.int32)
        lat = np.zeros(n, dtype=np.float64)
        wall = ctypes.c_double(0.0)
        t_seq = np.ascontiguousarray(batch.t_seq, dtype=np.uint8)
        q_seq = np.ascontiguousarray(batch.q_seq, dtype=np.uint8)
        t_off = np.ascontiguousarray(np.asarray(batch.t_off)[sel], dtype=np.int64)
        q_off = np.ascontiguousarray(np.asarray(batch.q_off)[sel], dtype=np.int64)
        t_len = np.ascontiguousarray(np.asarray(batch.t_len)[sel], dtype=np.int32)
        q_len = np.ascontiguousarray(np.asarray(batch.q_len)[sel], dtype=np.int32)
        _check(self.lib.ga_server_replay(self._h, t_seq.ctypes.data, t_off.ctypes.data, t_len.ctypes.data,
                                         q_seq.ctypes.data, q_off.ctypes.data, q_len.ctypes.data, arr.ctypes.data,
                                         n, res.ctypes.data, lat.ctypes.data, ctypes.byref(wall)),
               "ga_server_replay")
        return res, lat, float(wall.value)

    @property
    def batches(self) -> int:
        return int(self.lib.ga_server_batches(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.ga_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve_trace_native(batch, arrivals: np.ndarray, device: int = 0, pairs=None, **server_args):
    """As serve_trace, with the native server."""
    srv = NativeServer(batch.scoring, batch.w, batch.zdrop, device, **server_args)
    res, lat, wall = srv.replay(batch, arrivals, pairs)
    nb = srv.batches
    srv.close()
    return res, lat, wall, nb


def serve_trace(batch, arrivals: np.ndarray, device: int = 0, pairs=None, timeout_s: float = 60.0,
                **server_args):
    """Replay a request trace: request k (pair ``pairs[k]`` of ``batch``,
    pair k without ``pairs``) arrives at ``arrivals[k]`` seconds after the
    start. Returns (results [n, 7], latencies in seconds, wall seconds,
    batches launched); raises TimeoutError when requests stay in flight for
    ``timeout_s`` seconds with no batch finishing."""
    n = int(np.asarray(arrivals).shape[0])
    sel = np.arange(batch.n_pairs) if pairs is None else np.asarray(pairs, dtype=np.int64)
    if sel.shape[0] != n:
        raise ValueError("one arrival time per request")
    srv = Server(batch.scoring, batch.w, batch.zdrop, device, **server_args)
    results = np.zeros((n, 7), dtype=np.int32)
    t_arr = np.zeros(n)
    t_done = np.zeros(n)
    nxt = 0
    finished = 0
    t0 = time.perf_counter()
    progress = t0  # the last submission or collection
    while finished < n:
        now = time.perf_counter() - t0
        if not srv.idle and time.perf_counter() - progress > timeout_s:
            srv.close()
            raise TimeoutError(f"no batch finished in {timeout_s} s with requests in flight")
        while nxt < n and arrivals[nxt] <= now:
            t_arr[nxt] = t0 + arrivals[nxt]
            srv.submit(nxt, batch.target(int(sel[nxt])), batch.query(int(sel[nxt])), t_arr[nxt])
            nxt += 1
            progress = time.perf_counter()
        for rid, row, t in srv.step():
            results[rid] = row
            t_done[rid] = t
            finished += 1
            progress = time.perf_counter()
        if nxt < n and srv.idle:
            # nothing in flight: sleep until the next arrival (bounded)
            time.sleep(max(0.0, min(0.002, arrivals[nxt] - (time.perf_counter() - t0))))
        else:
            time.sleep(0.00005)
    wall = time.perf_counter() - t0
    batches = srv.batches
    srv.close()
    return results, t_done - t_arr, wall, batches


def offline(batch, device: int = 0, repeats: int = 3):
    """The same requests as one batch: (results, seconds per batch)."""
    torch = _torch()
    ctx = Context(device)
    packed = pack_batch(ctx, batch)
    out = ga_align_batch(ctx, packed, batch.scoring, batch.w, batch.zdrop)
    torch.cuda.synchronize()
    ctx.check()
    t0 = time.perf_counter()
    for _ in range(repeats):
        ga_align_batch(ctx, packed, batch.scoring, batch.w, batch.zdrop, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / repeats
    ctx.check()
    res = out.cpu().numpy()
    ctx.close()
    return res, dt


def serving_benchmark(requests: int = 20000, rates=(0.5, 0.8), duration=None, seed: int = 0,
                      python_loop: bool = False, log=None, **server_args):
    """Offline batch, saturated server and Poisson arrivals at fractions of
    the saturated throughput over the ``serving`` workload's request pool;
    returns one dict per rate (latency percentiles, throughput, whether every
    served result equals the offline batch's). ``duration``: seconds of
    arrivals per rate, cycling over the pool (default: the pool once)."""
    import seqgen

    say = log or (lambda msg: sys.stderr.write(msg + "\n"))
    batch = seqgen.make_workload("serving", n_pairs=requests, seed=seed)
    res_off, dt_off = offline(batch)
    cells_pool = count_cells(batch.t_len, batch.q_len, batch.w, res_off)
    cells = int(cells_pool.sum())
    say(f"[serve] offline: {batch.n_pairs} requests as one batch in {dt_off * 1e3:.1f} ms "
        f"({batch.n_pairs / dt_off:.0f} req/s, {cells / dt_off / 1e9:.1f} GCUPS)")
    # the server's own capacity: every request waiting at the start
    run = serve_trace if python_loop else serve_trace_native
    res_sat, lat_sat, wall_sat, nb_sat = run(batch, np.zeros(batch.n_pairs), **server_args)
    capacity = batch.n_pairs / wall_sat
    say(f"[serve] saturated: {wall_sat * 1e3:.1f} ms, {capacity:.0f} req/s, {nb_sat} batches, "
        f"{cells / wall_sat / 1e9:.1f} GCUPS")
    if not np.array_equal(res_sat, res_off):
        raise RuntimeError("served results differ from the offline batch")
    long_pool = batch.t_len + batch.q_len > 8000
    lines = []
    for frac in rates:
        qps = frac * capacity
        rng = np.random.default_rng([5, seed, 1])
        n_req = batch.n_pairs if duration is None else max(1, int(np.ceil(qps * duration)))
        arrivals = np.cumsum(rng.exponential(1.0 / qps, size=n_req))
        pairs = np.arange(n_req) % batch.n_pairs  # request k asks for pool pair k mod pool size
        res, lat, wall, nb = run(batch, arrivals, pairs=pairs, **server_args)
        same = bool(np.array_equal(res, res_off[pairs]))
        long_ = long_pool[pairs]
        req_cells = int(cells_pool[pairs].sum())
        line = {
            "metric": "serving latency", "unit": "ms", "qps": round(qps, 1), "rate_of_capacity": frac,
            "capacity_req_per_s": round(capacity, 1), "requests": n_req, "pool": batch.n_pairs,
            "served_req_per_s": round(n_req / wall, 1),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "p50_short_ms": round(float(np.percentile(lat[~long_], 50)) * 1e3, 3),
            "p99_short_ms": round(float(np.percentile(lat[~long_], 99)) * 1e3, 3),
            "p50_long_ms": round(float(np.percentile(lat[long_], 50)) * 1e3, 3) if long_.any() else None,
            "p99_long_ms": round(float(np.percentile(lat[long_], 99)) * 1e3, 3) if long_.any() else None,
            "gcups": round(req_cells / wall / 1e9, 3), "offline_gcups": round(cells / dt_off / 1e9, 3),
            "saturated_gcups": round(cells / wall_sat / 1e9, 3),
            "batches": nb, "wall_s": round(wall, 3), "same_as_offline": same,
            "graphs": bool(server_args.get("graphs", True)),
            "host_loop": "python" if python_loop else "native",
            "workload": "seqgen serving workload: 95% pairs of 100-1000 bp (5% errors), 5% of 10-25 kb "
                        "(1% errors + indels), w=500, Z=400, Poisson arrivals",
        }
        say(f"[serve] rate {frac}: {n_req} requests, p50 {line['p50_ms']} ms, p99 {line['p99_ms']} ms, "
            f"same as offline: {same}")
        lines.append(line)
        if not same:
            raise RuntimeError("served results differ from the offline batch")
    return lines


def main(argv=None):
    ap = argparse.ArgumentParser(description="serving benchmark (continuous batching)")
    ap.add_argument("--requests", type=int, default=20000)
    ap.add_argument("--rates", type=float, nargs="+", default=[0.5, 0.8],
                    help="arrival rates as fractions of the server's saturated throughput")
    ap.add_argument("--slots", type=int, default=2)
    ap.add_argument("--long-slots", type=int, default=1)
    ap.add_argument("--max-batch-pairs", type=int, default=256)
    ap.add_argument("--max-batch-bases", type=int, default=1_000_000)
    ap.add_argument("--long-batch-pairs", type=int, default=4096)
    ap.add_argument("--long-batch-bases", type=int, default=16_000_000)
    ap.add_argument("--no-graphs", action="store_true", help="enqueue each batch's steps eagerly")
    ap.add_argument("--python", action="store_true", help="drive the slots from the Python loop (Server) "
                    "instead of the native server")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--duration", type=float, default=None,
                    help="seconds of arrivals per rate, cycling over the request pool (default: "
                         "each rate serves the pool once)")
    args = ap.parse_args(argv)
    torch = _torch()
    torch.cuda.set_device(0)
    kw = dict(slots=args.slots, long_slots=args.long_slots, max_batch_pairs=args.max_batch_pairs,
              max_batch_bases=args.max_batch_bases, long_batch_pairs=args.long_batch_pairs,
              long_batch_bases=args.long_batch_bases, graphs=not args.no_graphs)
    try:
        lines = serving_benchmark(args.requests, args.rates, args.duration, args.seed, args.python, **kw)
    except RuntimeError as e:
        raise SystemExit(str(e))
    for line in lines:
        print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
