"""Continuous-batching request loop over the C ABI's server calls.

Frames (requests) of many streams arrive over time.  A stream's state stays
on the device from its admission to its last frame; streams are admitted in
order of their first arrival while their device bytes (``stream_bytes``) fit a
memory budget, and retired, freeing their bytes, once their last frame is
done.  Whenever fewer than ``depth`` launches are on the GPU and admitted
streams have frames waiting, one ``ddh_server_step`` advances every such
stream by its oldest waiting frame.  Launches go to one HIP stream and run in
order, so a frame arriving while others are on the GPU joins the next launch,
and a stream may have frames in consecutive launches.  A stream's frames are
processed in arrival order, and its numerics do not depend on which other
streams share a launch.

``Scheduler`` holds the host-side policy only (no device calls) and is tested
on the CPU; ``ServeLoop`` drives it against the device in real time.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field


@dataclass
class Request:
    """One frame of one stream."""
    t_arrival: float          # seconds from the start of the run
    key: object               # stream identity
    index: int                # frame index within its stream (0, 1, ...)
    last: bool                # the stream ends after this frame
    payload: object = None    # the device frame (opaque to the scheduler)
    t_admit: float | None = None  # when its stream was admitted (or its arrival, if later)
    t_done: float | None = None


@dataclass
class _StreamState:
    key: object
    nbytes: int
    queue: collections.deque = field(default_factory=collections.deque)
    admitted: bool = False
    next_index: int = 0       # next frame index to launch (arrival order is enforced)
    in_flight: int = 0
    finished: bool = False    # last frame launched


class Scheduler:
    """Admission by memory budget and per-launch frame selection."""

    def __init__(self, budget_bytes: int, max_batch: int):
        if budget_bytes <= 0 or max_batch <= 0:
            raise ValueError("budget and batch size must be positive")
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.used = 0
        self.streams: dict = {}
        self.waiting: collections.deque = collections.deque()  # keys not yet admitted, by first arrival
        self.order: list = []                                   # admitted keys, by admission

    def arrive(self, req: Request, nbytes: int) -> None:
        st = self.streams.get(req.key)
        if st is None:
            if nbytes > self.budget:
                raise ValueError(f"stream {req.key!r} needs {nbytes} bytes, more than the whole budget")
            st = self.streams[req.key] = _StreamState(req.key, int(nbytes))
            self.waiting.append(req.key)
        if st.finished:
            raise ValueError(f"frame after the last frame of stream {req.key!r}")
        if st.admitted:
            req.t_admit = req.t_arrival
        st.queue.append(req)

    def admit(self, now: float = 0.0) -> list:
        """Admit waiting streams in arrival order while they fit; a stream
        that does not fit blocks the ones behind it (no overtaking)."""
        newly = []
        while self.waiting:
            st = self.streams[self.waiting[0]]
            if self.used + st.nbytes > self.budget:
                break
            self.waiting.popleft()
            st.admitted = True
            self.used += st.nbytes
            self.order.append(st.key)
            for req in st.queue:
                req.t_admit = max(now, req.t_arrival)
            newly.append(st.key)
        return newly

    def next_batch(self) -> list:
        """The oldest waiting frame of every admitted stream that has one, at
        most max_batch of them, oldest first (max_batch = 1 gives the
        one-frame-at-a-time loop in arrival order)."""
        heads = sorted((self.streams[k].queue[0].t_arrival, i, k) for i, k in enumerate(self.order)
                       if self.streams[k].queue)
        batch = []
        for _, _, key in heads:
            st = self.streams[key]
            req = st.queue[0]
            if req.index != st.next_index:
                raise ValueError(f"stream {key!r}: frame {req.index} arrived before frame {st.next_index}")
            st.queue.popleft()
            st.next_index += 1
            st.in_flight += 1
            if req.last:
                st.finished = True
            batch.append(req)
            if len(batch) == self.max_batch:
                break
        return batch

    def complete(self, batch: list, t_done: float) -> list:
        """Mark a launch done; returns the keys of streams retired by it."""
        retired = []
        for req in batch:
            req.t_done = t_done
            st = self.streams[req.key]
            st.in_flight -= 1
            if st.finished and st.in_flight == 0 and not st.queue:
                self.used -= st.nbytes
                self.order.remove(st.key)
                del self.streams[st.key]
                retired.append(st.key)
        return retired

    def idle(self) -> bool:
        return not self.streams


class ServeLoop:
    """Runs a list of requests against the device in real time.

    make_stream(key) -> a ``Stream`` (called on admission; the stream is
    closed on retirement, after on_retire(key, stream) if given);
    nbytes(key) -> its device bytes.  Request payloads are device frames.
    Returns the requests with ``t_done`` set (seconds from the start; a
    launch's completion is seen by polling its HIP event).
    """

    def __init__(self, budget_bytes: int, max_batch: int = 64, depth: int = 2, plain: bool = False):
        self.budget = budget_bytes
        self.max_batch = max_batch
        self.depth = depth
        self.plain = plain  # one stream per launch, in arrival order (the one-at-a-time loop)

    def run(self, requests, make_stream, nbytes, on_retire=None):
        import torch
        import paper_2305_03284_amd as D
        reqs = sorted(requests, key=lambda r: (r.t_arrival, str(r.key), r.index))
        sched = Scheduler(self.budget, 1 if self.plain else self.max_batch)
        server = None if self.plain else D.Server(self.max_batch)
        live = {}
        inflight = collections.deque()
        nxt = 0
        t0 = time.perf_counter()
        try:
            while nxt < len(reqs) or not sched.idle():
                now = time.perf_counter() - t0
                while nxt < len(reqs) and reqs[nxt].t_arrival <= now:
                    r = reqs[nxt]
                    sched.arrive(r, nbytes(r.key))
                    nxt += 1
                # retire finished launches
                while inflight and inflight[0][0].query():
                    ev, batch = inflight.popleft()
                    t_done = time.perf_counter() - t0
                    for key in sched.complete(batch, t_done):
                        s = live.pop(key)
                        if on_retire is not None:
                            on_retire(key, s)
                        s.close()
                for key in sched.admit(time.perf_counter() - t0):
                    live[key] = make_stream(key)
                if len(inflight) < self.depth:
                    batch = sched.next_batch()
                    if batch:
                        streams = [live[r.key] for r in batch]
                        if self.plain:
                            streams[0].step(batch[0].payload)
                        else:
                            server.step(streams, [r.payload for r in batch])
                        ev = torch.cuda.Event()
                        ev.record()
                        inflight.append((ev, batch))
                        continue
                if inflight and (nxt >= len(reqs) or reqs[nxt].t_arrival > now):
                    # nothing to launch: wait a little for the GPU or the next arrival
                    time.sleep(2e-5)
        finally:
            torch.cuda.synchronize()
            for s in live.values():
                s.close()
            if server is not None:
                server.close()
        return reqs


def poisson_requests(keys, rate_hz: float, frames_per_stream: int, seed: int, start_spread_s: float = 0.0):
    """Frame arrival times: each stream starts at a uniform time in
    [0, start_spread_s) and then emits frames_per_stream frames by a Poisson
    process of rate rate_hz / len(keys) (so rate_hz is the aggregate while all
    streams are live)."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    per = rate_hz / len(keys)
    out = []
    for key in keys:
        t = rng.uniform(0.0, start_spread_s) if start_spread_s > 0 else 0.0
        for n in range(frames_per_stream):
            t += rng.exponential(1.0 / per)
            out.append(Request(t, key, n, n == frames_per_stream - 1))
    return out


def latency_stats(reqs) -> dict:
    """Frame latency from arrival, service latency from admission (differs
    only for frames that waited for their stream's admission), throughput."""
    import numpy as np
    lat = np.array([r.t_done - r.t_arrival for r in reqs])
    svc = np.array([r.t_done - r.t_admit for r in reqs])
    span = max(r.t_done for r in reqs) - min(r.t_arrival for r in reqs)
    return {"frames": len(reqs), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "service_p50_ms": float(np.percentile(svc, 50) * 1e3), "service_p99_ms": float(np.percentile(svc, 99) * 1e3),
            "frames_per_s": len(reqs) / span}
