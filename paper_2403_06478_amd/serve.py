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
import dataclasses
import json
import sys
import time
from typing import List, Optional

import numpy as np

from . import (Context, _check, _stream_handle, _torch, count_cells, ga_align_batch, load_library,
               pack_batch)


@dataclasses.dataclass
class _Request:
    rid: int
    target: bytes
    query: bytes
    t_arrival: float


class _HostBatch:
    """The minimal batch interface ``pack_batch`` reads (ASCII buffers)."""

    def __init__(self, reqs: List[_Request]):
        tl = np.array([len(r.target) for r in reqs], dtype=np.int32)
        ql = np.array([len(r.query) for r in reqs], dtype=np.int32)
        self.t_len, self.q_len = tl, ql
        self.t_off = np.zeros(len(reqs), dtype=np.int64)
        self.q_off = np.zeros(len(reqs), dtype=np.int64)
        if len(reqs) > 1:
            self.t_off[1:] = np.cumsum(tl[:-1], dtype=np.int64)
            self.q_off[1:] = np.cumsum(ql[:-1], dtype=np.int64)
        self.t_seq = np.frombuffer(b"".join(r.target for r in reqs), dtype=np.uint8).copy()
        self.q_seq = np.frombuffer(b"".join(r.query for r in reqs), dtype=np.uint8).copy()
        self.n_pairs = len(reqs)


class _Slot:
    def __init__(self, device: int):
        torch = _torch()
        self.ctx = Context(device)
        self.stream = torch.cuda.Stream(device=device)  # default priority
        self.reqs: Optional[List[_Request]] = None
        self.event = None
        self.keep = None
        self.host_out = None

    @property
    def busy(self) -> bool:
        return self.reqs is not None

    def launch(self, reqs: List[_Request], scoring: dict, w: int, Z: int):
        torch = _torch()
        hb = _HostBatch(reqs)
        with torch.cuda.stream(self.stream):
            packed = pack_batch(self.ctx, hb, self.stream)
            out = ga_align_batch(self.ctx, packed, scoring, w, Z, stream=self.stream)
            host_out = torch.empty(out.shape, dtype=out.dtype, pin_memory=True)
            host_out.copy_(out, non_blocking=True)
            self.event = torch.cuda.Event()
            self.event.record(self.stream)
        self.keep = (packed, out)
        self.host_out = host_out
        self.reqs = reqs

    def poll(self):
        """(requests, results) once the batch has completed, else None."""
        if self.reqs is None or not self.event.query():
            return None
        _check(load_library().ga_context_check(self.ctx.handle, _stream_handle(self.stream)),
               "ga_context_check")
        reqs, res = self.reqs, self.host_out.numpy().copy()
        self.reqs = self.event = self.keep = self.host_out = None
        return reqs, res


class Server:
    """Continuous batching over ``slots`` concurrent device batches.

    ``max_batch_pairs`` and ``max_batch_bases`` bound one batch; a request
    longer than ``max_batch_bases`` alone still forms a batch of its own."""

    def __init__(self, scoring: dict, w: int, Z: int, device: int = 0, slots: int = 4,
                 max_batch_pairs: int = 512, max_batch_bases: int = 2_000_000):
        self.scoring, self.w, self.Z = dict(scoring), int(w), int(Z)
        self.slots = [_Slot(device) for _ in range(slots)]
        self.max_batch_pairs = int(max_batch_pairs)
        self.max_batch_bases = int(max_batch_bases)
        self.pending = collections.deque()
        self.batches = 0

    def submit(self, rid: int, target: bytes, query: bytes, t_arrival: Optional[float] = None):
        self.pending.append(_Request(rid, target, query,
                                     time.perf_counter() if t_arrival is None else t_arrival))

    def _take_batch(self) -> List[_Request]:
        reqs, bases = [], 0
        while self.pending and len(reqs) < self.max_batch_pairs:
            r = self.pending[0]
            size = len(r.target) + len(r.query)
            if reqs and bases + size > self.max_batch_bases:
                break
            reqs.append(self.pending.popleft())
            bases += size
        return reqs

    def step(self):
        """Collect finished batches, then start batches on free slots.
        Returns [(rid, result row, t_done)] for the requests that finished."""
        done = []
        for slot in self.slots:
            got = slot.poll()
            if got is not None:
                t = time.perf_counter()
                reqs, res = got
                done.extend((r.rid, res[k], t) for k, r in enumerate(reqs))
        for slot in self.slots:
            if not self.pending:
                break
            if not slot.busy:
                slot.launch(self._take_batch(), self.scoring, self.w, self.Z)
                self.batches += 1
        return done

    @property
    def idle(self) -> bool:
        return not self.pending and not any(s.busy for s in self.slots)

    def close(self):
        for s in self.slots:
            s.ctx.close()


def serve_trace(batch, arrivals: np.ndarray, slots: int = 4, max_batch_pairs: int = 512,
                max_batch_bases: int = 2_000_000, device: int = 0):
    """Replay a request trace: request k (pair k of ``batch``) arrives at
    ``arrivals[k]`` seconds after the start. Returns (results [n, 7],
    latencies in seconds, wall seconds, batches launched)."""
    n = batch.n_pairs
    srv = Server(batch.scoring, batch.w, batch.zdrop, device, slots, max_batch_pairs, max_batch_bases)
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
    ap.add_argument("--requests", type=int, default=6000)
    ap.add_argument("--rates", type=float, nargs="+", default=[0.5, 0.8],
                    help="arrival rates as fractions of the offline capacity")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--max-batch-pairs", type=int, default=512)
    ap.add_argument("--max-batch-bases", type=int, default=2_000_000)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)
    torch = _torch()
    torch.cuda.set_device(0)
    batch = seqgen.make_config(5, n_pairs=args.requests, seed=args.seed)
    res_off, dt_off = offline(batch)
    cells = int(count_cells(batch.t_len, batch.q_len, batch.w, res_off).sum())
    capacity = batch.n_pairs / dt_off
    sys.stderr.write(f"[serve] offline: {batch.n_pairs} requests in {dt_off * 1e3:.1f} ms "
                     f"({capacity:.0f} req/s, {cells / dt_off / 1e9:.1f} GCUPS)\n")
    for frac in args.rates:
        qps = frac * capacity
        rng = np.random.default_rng([5, args.seed, 1])
        arrivals = np.cumsum(rng.exponential(1.0 / qps, size=batch.n_pairs))
        res, lat, wall, nb = serve_trace(batch, arrivals, args.slots, args.max_batch_pairs,
                                         args.max_batch_bases)
        same = bool(np.array_equal(res, res_off))
        long_ = batch.t_len >= 10000
        line = {
            "metric": "serving latency", "unit": "ms", "qps": round(qps, 1), "rate_of_capacity": frac,
            "requests": batch.n_pairs, "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "p50_short_ms": round(float(np.percentile(lat[~long_], 50)) * 1e3, 3),
            "p99_long_ms": round(float(np.percentile(lat[long_], 99)) * 1e3, 3) if long_.any() else None,
            "gcups": round(cells / wall / 1e9, 3), "offline_gcups": round(cells / dt_off / 1e9, 3),
            "batches": nb, "slots": args.slots, "wall_s": round(wall, 3), "same_as_offline": same,
            "workload": "seqgen workload 5: 95% pairs of 100-1000 bp (5% errors), 5% of 10-25 kb "
                        "(1% errors + indels), w=500, Z=400, Poisson arrivals",
        }
        print(json.dumps(line), flush=True)
        if not same:
            raise SystemExit("served results differ from the offline batch")


if __name__ == "__main__":
    main()
