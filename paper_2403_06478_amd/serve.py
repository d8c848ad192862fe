"""Continuous-batching serving loop over the C ABI.

Requests (one target/query pair each) arrive over time. The server keeps a
FIFO of admitted requests and a few execution slots; each slot owns a
context (its own device workspace) and a HIP stream. Whenever a slot is
free, the requests waiting at that moment form its next batch, up to a pair
count and a memory footprint (bases staged on the device), and the batch is
packed, aligned and copied back on the slot's stream. Slots run
concurrently, so requests that arrive while other batches are on the GPU are
admitted as soon as a slot frees up and their work overlaps on the device
with the batches already running. A request's latency runs from its arrival
to the moment the host sees its batch complete.

Every step of the alignment runs in the HIP library; this module only
schedules batches and moves bytes.

``python -m paper_2403_06478_amd.serve`` runs the serving benchmark: the
request mix of ``seqgen`` workload 5 with Poisson arrivals at given
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

from . import (Batch, Context, _check, _stream_handle, _torch, count_cells, ga_align_batch,
               load_library, pack_batch, scoring_struct)


@dataclasses.dataclass
class _Request:
    rid: int
    target: bytes
    query: bytes
    t_arrival: float


class _Slot:
    """One execution slot: a context (own device workspace), a HIP stream,
    and staging buffers sized once for the largest batch -- pinned host
    buffers for the request bytes and results, device buffers for the packed
    streams -- so a batch allocates nothing (an allocation can synchronise
    the device and stall every other slot).

    With ``graphs`` the device steps of a batch (packing both sides and the
    alignment) are one captured HIP graph, launched once per batch: every
    batch is presented at the slot's capacity (the unused pair entries are
    empty pairs, which the planner finishes at once, and the packed streams
    are declared at their full capacity), so the same graph serves every
    batch; only the request bytes, offsets and lengths are copied in before
    the launch and the used results copied out after it."""

    # longest sequence a captured batch declares (the bound its range guard checks)
    GRAPH_MAX_LEN = 1 << 20

    def __init__(self, device: int, max_pairs: int, max_bases: int, scoring: dict, w: int, Z: int,
                 graphs: bool = True):
        self.lib = load_library()
        self.ctx = Context(device)
        # one stream per slot: the slots already overlap, and more streams
        # than the GPU's hardware queues would serialise unrelated batches
        self.ctx.set_lanes(1)
        self.stream = _torch().cuda.Stream(device=device)  # default priority
        self.device = device
        self.scoring, self.w, self.Z = dict(scoring), int(w), int(Z)
        self.graphs = bool(graphs)
        self.graph = None
        self.max_pairs = self.max_bases = 0
        self._size(max_pairs, max_bases)
        self.reqs: Optional[List[_Request]] = None
        self.event = None

    def _size(self, max_pairs: int, max_bases: int):
        """(Re)allocate the staging buffers for batches of up to max_pairs
        pairs and max_bases bases per side (and drop the captured graph,
        which names the old buffers). Only an oversized request makes a slot
        grow after start."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        self.graph = None
        self.max_pairs, self.max_bases = P, B = int(max(max_pairs, 1)), int(max(max_bases, 1))
        self.W = W = B // 16 + P + 1  # 2-bit words of one side: at most sum of ceil(len / 16)
        pin = dict(pin_memory=True)
        self.h_ascii = [torch.empty(B, dtype=torch.uint8, **pin) for _ in range(2)]
        # unused entries stay empty pairs (offset 0, length 0)
        self.h_off = [torch.zeros(P, dtype=torch.int64, **pin) for _ in range(2)]
        self.h_len = [torch.zeros(P, dtype=torch.int32, **pin) for _ in range(2)]
        self.h_out = torch.empty((P, 7), dtype=torch.int32, **pin)
        self.d_ascii = [torch.zeros(B, dtype=torch.uint8, device=dev) for _ in range(2)]
        self.d_off = [torch.zeros(P, dtype=torch.int64, device=dev) for _ in range(2)]
        self.d_len = [torch.zeros(P, dtype=torch.int32, device=dev) for _ in range(2)]
        self.d_words = [torch.zeros(W, dtype=torch.int32, device=dev) for _ in range(2)]
        self.d_woff = [torch.zeros(P, dtype=torch.int64, device=dev) for _ in range(2)]
        self.d_nmask = [torch.zeros((W + 1) // 2, dtype=torch.int32, device=dev) for _ in range(2)]
        self.d_out = torch.empty((P, 7), dtype=torch.int32, device=dev)
        torch.cuda.synchronize(self.device)

    def _device_steps(self, st: int, n: int, nwords, max_len: int):
        """Pack both sides and align n pairs, all enqueued on stream st."""
        for side in range(2):
            _check(self.lib.ga_pack(self.ctx.handle, self.d_ascii[side].data_ptr(), self.d_off[side].data_ptr(),
                                    self.d_len[side].data_ptr(), n, nwords[side], self.d_words[side].data_ptr(),
                                    self.d_woff[side].data_ptr(), self.d_nmask[side].data_ptr(), st), "ga_pack")
        bt = Batch()
        bt.n_pairs = n
        bt.t_words_dev, bt.t_nwords = self.d_words[0].data_ptr(), nwords[0]
        bt.q_words_dev, bt.q_nwords = self.d_words[1].data_ptr(), nwords[1]
        bt.t_off_dev, bt.q_off_dev = self.d_woff[0].data_ptr(), self.d_woff[1].data_ptr()
        bt.t_len_dev, bt.q_len_dev = self.d_len[0].data_ptr(), self.d_len[1].data_ptr()
        bt.t_nmask_dev, bt.q_nmask_dev = self.d_nmask[0].data_ptr(), self.d_nmask[1].data_ptr()
        bt.max_len = int(max_len)
        sc = scoring_struct(self.scoring)
        _check(self.lib.ga_align_batch(self.ctx.handle, ctypes.byref(bt), ctypes.byref(sc), self.w, self.Z,
                                       self.d_out.data_ptr(), st), "ga_align_batch")

    def _capture(self):
        """Capture the capacity-shaped device steps (after one eager run on
        the empty staging, which sizes the context's workspace)."""
        torch = _torch()
        shape = (self.max_pairs, [self.W, self.W], min(self.max_bases, self.GRAPH_MAX_LEN))
        with torch.cuda.stream(self.stream):
            self._device_steps(_stream_handle(self.stream), *shape)
        self.stream.synchronize()
        _check(self.lib.ga_context_check(self.ctx.handle, _stream_handle(self.stream)), "ga_context_check")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=self.stream):
            self._device_steps(_stream_handle(torch.cuda.current_stream()), *shape)
        self.graph = g

    @property
    def busy(self) -> bool:
        return self.reqs is not None

    def launch(self, reqs: List[_Request]):
        torch = _torch()
        n = len(reqs)
        lens = [np.array([len(r.target) for r in reqs], dtype=np.int32),
                np.array([len(r.query) for r in reqs], dtype=np.int32)]
        bases = max(int(lens[0].sum()), int(lens[1].sum()))
        if n > self.max_pairs or bases > self.max_bases:
            self._size(max(n, self.max_pairs), max(bases, self.max_bases))
        max_len = int(max(lens[0].max(initial=0), lens[1].max(initial=0)))
        use_graph = self.graphs and max_len <= self.GRAPH_MAX_LEN
        if use_graph and self.graph is None:
            self._capture()
        P = self.max_pairs if use_graph else n
        with torch.cuda.stream(self.stream):
            for side in range(2):
                seqs = b"".join(r.target if side == 0 else r.query for r in reqs)
                off = np.zeros(n, dtype=np.int64)
                off[1:] = np.cumsum(lens[side][:-1], dtype=np.int64)
                self.h_ascii[side].numpy()[:len(seqs)] = np.frombuffer(seqs, dtype=np.uint8)
                h_off, h_len = self.h_off[side].numpy(), self.h_len[side].numpy()
                h_off[:n] = off
                h_len[:n] = lens[side]
                h_off[n:P] = 0
                h_len[n:P] = 0
                nb = max(len(seqs), 1)
                self.d_ascii[side][:nb].copy_(self.h_ascii[side][:nb], non_blocking=True)
                self.d_off[side][:P].copy_(self.h_off[side][:P], non_blocking=True)
                self.d_len[side][:P].copy_(self.h_len[side][:P], non_blocking=True)
            if use_graph:
                self.graph.replay()
            else:
                nwords = [int(self.lib.ga_pack_words(l.ctypes.data, n)) for l in lens]
                self._device_steps(_stream_handle(self.stream), n, nwords, max_len)
            self.h_out[:n].copy_(self.d_out[:n], non_blocking=True)
            self.event = torch.cuda.Event()
            self.event.record(self.stream)
        self.reqs = reqs

    def poll(self):
        """(requests, results) once the batch has completed, else None."""
        if self.reqs is None or not self.event.query():
            return None
        _check(self.lib.ga_context_check(self.ctx.handle, _stream_handle(self.stream)), "ga_context_check")
        reqs = self.reqs
        res = self.h_out.numpy()[:len(reqs)].copy()
        self.reqs = self.event = None
        return reqs, res


class Server:
    """Continuous batching over concurrent device batches, in two lanes.

    A request whose bases (target + query) exceed ``long_bases`` goes to the
    long lane, every other request to the short lane, so short requests never
    wait behind a long pair's sweep. Each lane has its own FIFO and slots
    (``slots`` short, ``long_slots`` long). A short batch holds up to
    ``max_batch_pairs`` pairs and ``max_batch_bases`` bases; a long batch up
    to ``long_batch_pairs`` pairs and ``long_batch_bases`` bases (a long pair
    runs on one workgroup for the whole of its sweep, so a long batch should
    take every long request waiting). A request larger than its lane's base limit still forms a batch
    of its own. Each slot's staging is sized once, at start, for its largest
    batch.

    HIP spreads streams over a few hardware queues (four by default) and the
    kernels of streams that share a queue run one after another, so a short
    batch would wait behind a long sweep; the defaults keep the slot streams
    at three."""

    def __init__(self, scoring: dict, w: int, Z: int, device: int = 0, slots: int = 2,
                 long_slots: int = 1, max_batch_pairs: int = 256, max_batch_bases: int = 1_000_000,
                 long_bases: int = 8000, long_batch_pairs: int = 4096, long_batch_bases: int = 16_000_000,
                 graphs: bool = True):
        self.scoring, self.w, self.Z = dict(scoring), int(w), int(Z)
        self.pairs = [int(max_batch_pairs), int(long_batch_pairs)]
        self.limits = [int(max_batch_bases), int(long_batch_bases)]
        self.lanes = [[_Slot(device, self.pairs[k], self.limits[k], scoring, w, Z, graphs) for _ in range(n)]
                      for k, n in enumerate((slots, long_slots))]
        self.long_bases = int(long_bases)
        self.pending = [collections.deque(), collections.deque()]
        self.batches = 0
        self._warm(device)

    def _warm(self, device: int):
        """Run one full-size batch through every slot so no later batch
        grows a workspace (which would synchronise the device). The warm-up
        pairs put the lane's bases in the targets and one base in each
        query, so their sweep stops at the band's edge (or, unbanded, after
        at most a few thousand anti-diagonals)."""
        torch = _torch()
        rng = np.random.default_rng(0)
        acgt = np.frombuffer(b"ACGT", dtype=np.uint8)
        for lane, P, limit in zip(self.lanes, self.pairs, self.limits):
            L = max(1, limit // P - 1)
            if self.w < 0:
                L = min(L, 4000)
            seq = rng.choice(acgt, L).tobytes()
            reqs = [_Request(-1, seq, b"A", 0.0) for _ in range(P)]
            for slot in lane:
                slot.launch(reqs)
        torch.cuda.synchronize(device)
        for lane in self.lanes:
            for slot in lane:
                slot.poll()

    def submit(self, rid: int, target: bytes, query: bytes, t_arrival: Optional[float] = None):
        lane = 1 if len(target) + len(query) > self.long_bases else 0
        self.pending[lane].append(_Request(rid, target, query,
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
        """Collect finished batches, then start batches on free slots.
        Returns [(rid, result row, t_done)] for the requests that finished."""
        done = []
        for lane in self.lanes:
            for slot in lane:
                got = slot.poll()
                if got is not None:
                    t = time.perf_counter()
                    reqs, res = got
                    done.extend((r.rid, res[k], t) for k, r in enumerate(reqs))
        for lane, q, P, limit in zip(self.lanes, self.pending, self.pairs, self.limits):
            for slot in lane:
                if not q:
                    break
                if not slot.busy:
                    slot.launch(self._take_batch(q, P, limit))
                    self.batches += 1
        return done

    @property
    def idle(self) -> bool:
        return not any(self.pending) and not any(s.busy for lane in self.lanes for s in lane)

    def close(self):
        for lane in self.lanes:
            for s in lane:
                s.ctx.close()


def serve_trace(batch, arrivals: np.ndarray, device: int = 0, **server_args):
    """Replay a request trace: request k (pair k of ``batch``) arrives at
    ``arrivals[k]`` seconds after the start. Returns (results [n, 7],
    latencies in seconds, wall seconds, batches launched)."""
    n = batch.n_pairs
    srv = Server(batch.scoring, batch.w, batch.zdrop, device, **server_args)
    results = np.zeros((n, 7), dtype=np.int32)
    t_arr = np.zeros(n)
    t_done = np.zeros(n)
    nxt = 0
    finished = 0
    t0 = time.perf_counter()
    while finished < n:
        now = time.perf_counter() - t0
        while nxt < n and arrivals[nxt] <= now:
            t_arr[nxt] = t0 + arrivals[nxt]
            srv.submit(nxt, batch.target(nxt), batch.query(nxt), t_arr[nxt])
            nxt += 1
        for rid, row, t in srv.step():
            results[rid] = row
            t_done[rid] = t
            finished += 1
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


def main(argv=None):
    import seqgen

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
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)
    torch = _torch()
    torch.cuda.set_device(0)
    batch = seqgen.make_config(5, n_pairs=args.requests, seed=args.seed)
    kw = dict(slots=args.slots, long_slots=args.long_slots, max_batch_pairs=args.max_batch_pairs,
              max_batch_bases=args.max_batch_bases, long_batch_pairs=args.long_batch_pairs,
              long_batch_bases=args.long_batch_bases, graphs=not args.no_graphs)
    res_off, dt_off = offline(batch)
    cells = int(count_cells(batch.t_len, batch.q_len, batch.w, res_off).sum())
    sys.stderr.write(f"[serve] offline: {batch.n_pairs} requests as one batch in {dt_off * 1e3:.1f} ms "
                     f"({batch.n_pairs / dt_off:.0f} req/s, {cells / dt_off / 1e9:.1f} GCUPS)\n")
    # the server's own capacity: every request waiting at the start
    res_sat, lat_sat, wall_sat, nb_sat = serve_trace(batch, np.zeros(batch.n_pairs), **kw)
    capacity = batch.n_pairs / wall_sat
    sys.stderr.write(f"[serve] saturated: {wall_sat * 1e3:.1f} ms, {capacity:.0f} req/s, {nb_sat} batches, "
                     f"{cells / wall_sat / 1e9:.1f} GCUPS\n")
    if not np.array_equal(res_sat, res_off):
        raise SystemExit("served results differ from the offline batch")
    long_ = batch.t_len + batch.q_len > 8000
    for frac in args.rates:
        qps = frac * capacity
        rng = np.random.default_rng([5, args.seed, 1])
        arrivals = np.cumsum(rng.exponential(1.0 / qps, size=batch.n_pairs))
        res, lat, wall, nb = serve_trace(batch, arrivals, **kw)
        same = bool(np.array_equal(res, res_off))
        line = {
            "metric": "serving latency", "unit": "ms", "qps": round(qps, 1), "rate_of_capacity": frac,
            "capacity_req_per_s": round(capacity, 1), "requests": batch.n_pairs,
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "p50_short_ms": round(float(np.percentile(lat[~long_], 50)) * 1e3, 3),
            "p99_short_ms": round(float(np.percentile(lat[~long_], 99)) * 1e3, 3),
            "p50_long_ms": round(float(np.percentile(lat[long_], 50)) * 1e3, 3) if long_.any() else None,
            "p99_long_ms": round(float(np.percentile(lat[long_], 99)) * 1e3, 3) if long_.any() else None,
            "gcups": round(cells / wall / 1e9, 3), "offline_gcups": round(cells / dt_off / 1e9, 3),
            "saturated_gcups": round(cells / wall_sat / 1e9, 3),
            "batches": nb, "wall_s": round(wall, 3), "same_as_offline": same, "graphs": not args.no_graphs,
            "workload": "seqgen workload 5: 95% pairs of 100-1000 bp (5% errors), 5% of 10-25 kb "
                        "(1% errors + indels), w=500, Z=400, Poisson arrivals",
        }
        print(json.dumps(line), flush=True)
        if not same:
            raise SystemExit("served results differ from the offline batch")


if __name__ == "__main__":
    main()
