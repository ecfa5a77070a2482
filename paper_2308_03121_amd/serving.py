"""Continuous-batching server over the C-ABI batch call.

Clip streams arrive over time; each one asks for admission with its device footprint
(`nv_stream_footprint` plus a share of the batch workspace) and waits in the
admission queue while the HBM budget is used up.  Admitted streams keep their overlap
frame (features, pixels, luma, histogram) on the device between batches.  Every
scheduling step gathers the frames that have arrived on all admitted streams and runs
them as one `nv_enhance_batch` call, so a stream that arrives while a batch is on the
GPU joins the very next batch (iteration-level batching, not a queue of whole clips).
Per group the latency runs from the arrival of the frame that closes the group to the
completion of the batch that emitted it.

The executor holds one network context per colourspace and serves each stream with the
network trained for the stream's colourspace (matrix and range), as the paper's
framework loads the network for the clip's colourspace (section 3.1); a stream whose
colourspace has no network is rejected at admission.

The scheduler is host logic; the executor (`GpuExecutor`) is the only part that
touches the device, so the scheduling rules can be exercised with another executor.
"""
from __future__ import annotations

import heapq
import math
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class StreamSpec:
    """One synthetic clip stream: format, frame arrival times, scene starts."""
    sid: int
    width: int
    height: int
    bits: int
    chroma: int
    arrivals: list            # seconds after the start of the run, one per frame
    scene_starts: list = field(default_factory=list)
    matrix: int = 709         # colourspace: BT.601 / 709 / 2020 matrix, full range, centre siting
    full: bool = False
    centre: bool = False

    @property
    def n_frames(self) -> int:
        return len(self.arrivals)


def poisson_workload(n_streams=16, rate_total=40.0, sizes=((960, 540), (1920, 1080)), bits=(8, 10),
                     length=(30, 300), cut_every=(10, 60), start_mean=0.4, seed=3, max_time=None):
    """Streams drawn uniformly over sizes x bit depths (4:2:0), lengths U{length}, scene
    cuts every U{cut_every} frames; frames of each stream arrive as a Poisson process of
    rate rate_total / n_streams, stream starts staggered by Exp(start_mean)."""
    rng = np.random.default_rng(seed)
    per = rate_total / n_streams
    specs, start = [], 0.0
    for sid in range(n_streams):
        start += rng.exponential(start_mean)
        w, h = sizes[rng.integers(len(sizes))]
        b = int(bits[rng.integers(len(bits))])
        n = int(rng.integers(length[0], length[1] + 1))
        t, arr = start, []
        for _ in range(n):
            arr.append(t)
            t += rng.exponential(1.0 / per)
        if max_time is not None:
            arr = [a for a in arr if a < max_time] or arr[:1]
        cuts, c = [], 0
        while True:
            c += int(rng.integers(cut_every[0], cut_every[1] + 1))
            if c >= len(arr):
                break
            cuts.append(c)
        specs.append(StreamSpec(sid, int(w), int(h), b, 420, arr, cuts))
    return specs


@dataclass
class GroupRecord:
    sid: int
    index: int                # group index within its stream (= output pair index)
    ready: float              # arrival time of the frame that closes the group
    done: float = math.nan
    out: list | None = None   # output frames when kept


@dataclass
class _Live:
    spec: StreamSpec
    handle: object
    next_frame: int = 0       # next frame to submit
    groups_emitted: int = 0
    ended: bool = False
    bytes: int = 0


class Server:
    """Scheduling loop.  executor must provide open(spec) -> (handle, bytes),
    submit(list of (handle, spec, frame indices, end)) -> ticket (outputs per request),
    poll(ticket) -> bool, outputs(ticket), close(handle), now()."""

    def __init__(self, executor, hbm_budget: int, max_frames=256, max_groups=512, max_chain=16,
                 keep_outputs=False, max_batch_px=None):
        self.ex = executor
        self.budget = hbm_budget
        self.max_frames, self.max_groups, self.max_chain = max_frames, max_groups, max_chain
        # bound on the LR pixels of the groups of one batch (their device workspace)
        self.max_batch_px = max_batch_px
        self.keep = keep_outputs
        self.used = 0
        self.admitted: dict[int, _Live] = {}
        self.waiting: list = []      # admission queue (arrival order)
        self.records: list[GroupRecord] = []
        self.rejected = 0
        self.admissions = []         # (sid, time admitted)
        self.batches = 0
        self.batch_sizes = []

    def _try_admit(self, now):
        while self.waiting:
            spec = self.waiting[0]
            need = self.ex.footprint(spec)
            if need > self.budget:
                self.waiting.pop(0)
                self.rejected += 1
                continue
            if self.used + need > self.budget:
                break
            self.waiting.pop(0)
            handle = self.ex.open(spec)
            self.admitted[spec.sid] = _Live(spec, handle, bytes=need)
            self.used += need
            self.admissions.append((spec.sid, now))

    def run(self, specs, time_scale=1.0):
        """Run the workload in real time (arrival times scaled by time_scale)."""
        self._px = {s.sid: s.width * s.height for s in specs}
        self._first = {s.sid: s.arrivals[0] for s in specs}
        pending = sorted(specs, key=lambda s: s.arrivals[0])
        t0 = self.ex.now()
        clock = lambda: (self.ex.now() - t0) / time_scale
        inflight = []           # (ticket, [(live, group records)])
        arrivals = [(s.arrivals[0], s.sid, s) for s in pending]
        heapq.heapify(arrivals)
        while arrivals or self.waiting or self.admitted or inflight:
            now = clock()
            while arrivals and arrivals[0][0] <= now:
                self.waiting.append(heapq.heappop(arrivals)[2])
            self._try_admit(now)
            # completions
            still = []
            for ticket, recs in inflight:
                if self.ex.poll(ticket):
                    tdone = clock()
                    outs = self.ex.outputs(ticket) if self.keep else None
                    for k, (live, rlist) in enumerate(recs):
                        for j, r in enumerate(rlist):
                            r.done = tdone
                            if outs is not None:
                                r.out = outs[k][2 * j:2 * j + 2]
                    self.ex.release(ticket)
                else:
                    still.append((ticket, recs))
            inflight = still
            # streams whose last group has completed leave and free their memory
            for sid in [sid for sid, lv in self.admitted.items() if lv.ended]:
                lv = self.admitted[sid]
                if all(not any(l is lv for l, _ in recs) for _, recs in inflight):
                    self.ex.close(lv.handle)
                    self.used -= lv.bytes
                    del self.admitted[sid]
            self._try_admit(now)
            # one batch of everything that has arrived
            reqs, recs, nf, ng, npx = [], [], 0, 0, 0
            for lv in self.admitted.values():
                if lv.ended:
                    continue
                spec = lv.spec
                j0, j = lv.next_frame, lv.next_frame
                gpx = spec.width * spec.height
                while j < spec.n_frames and spec.arrivals[j] <= now and j - j0 < self.max_chain:
                    if self.max_batch_px is not None and npx + gpx * (j + 1 - j0) > self.max_batch_px \
                            and (reqs or j > j0):
                        break
                    j += 1
                if j == j0:
                    continue
                end = j == spec.n_frames
                emit = (j - j0) - (1 if j0 == 0 else 0) + (1 if end else 0)
                if nf + (j - j0) > self.max_frames or ng + emit > self.max_groups:
                    continue
                rl = []
                for f in range(max(j0, 1), j):
                    rl.append(GroupRecord(spec.sid, f - 1, spec.arrivals[f]))
                if end:
                    rl.append(GroupRecord(spec.sid, spec.n_frames - 1, spec.arrivals[-1]))
                reqs.append((lv.handle, spec, list(range(j0, j)), end))
                recs.append((lv, rl))
                self.records += rl
                lv.next_frame = j
                lv.ended = end
                nf += j - j0
                ng += emit
                npx += gpx * emit
            if reqs:
                inflight.append((self.ex.submit(reqs), recs))
                self.batches += 1
                self.batch_sizes.append(ng)
                continue
            # nothing to do right now: wait for the next event
            nxt = [a[0] for a in arrivals[:1]]
            for lv in self.admitted.values():
                if not lv.ended and lv.next_frame < lv.spec.n_frames:
                    nxt.append(lv.spec.arrivals[lv.next_frame])
            if inflight:
                self.ex.wait_any([t for t, _ in inflight], 0.002)
            elif nxt:
                time.sleep(max(0.0, min(min(nxt) - clock(), 0.05)) * time_scale)
        return self.report(clock())

    def report(self, elapsed):
        lat = np.array([r.done - r.ready for r in self.records if not math.isnan(r.done)])
        mpix = sum(2 * 4 * self._spec_px(r.sid) for r in self.records) / 1e6
        return {
            "groups": len(self.records),
            "elapsed_s": elapsed,
            "output_mpix_per_s": mpix / elapsed if elapsed > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1000) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1000) if lat.size else None,
            "max_ms": float(lat.max() * 1000) if lat.size else None,
            "batches": self.batches,
            "mean_groups_per_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "admitted": len(self.admissions),
            "rejected": self.rejected,
            # time from a stream's first frame to its admission (waits for HBM budget)
            "admission_waited": int(sum(1 for sid, t in self.admissions if t - self._first.get(sid, t) > 1e-3)),
            "admission_wait_max_ms": float(max([1000 * (t - self._first.get(sid, t)) for sid, t in self.admissions]
                                               or [0.0])),
        }

    def _spec_px(self, sid):
        return self._px.get(sid, 0)


def torch_float32():
    import torch
    return torch.float32


def colourspace_of(obj):
    """(matrix, full range) of a stream spec or of a network context."""
    if hasattr(obj, "colourspace"):
        return tuple(obj.colourspace)
    return (int(obj.matrix), bool(obj.full))


def select_context(ctxs, spec):
    """The context whose network was trained for the stream's colourspace, or None.
    ctxs: one context, or a mapping (matrix, full) -> context."""
    key = colourspace_of(spec)
    if isinstance(ctxs, dict):
        return ctxs.get(key)
    return ctxs if colourspace_of(ctxs) == key else None


# Footprint of a stream no network can serve: larger than any budget, so the server
# rejects it at admission.
UNSERVABLE = 1 << 62


class GpuExecutor:
    """Executor over the library: one context per colourspace (a context or a mapping
    (matrix, full) -> context), one HIP stream, frames from a device bank.  Each batch
    step runs one nv_enhance_batch call per context with requests.  Streams that leave
    go to a pool per format and are reset for the next stream of that format, so
    serving never frees or allocates stream memory (a free would synchronise the device
    and stall the batches in flight)."""

    def __init__(self, ctx, frame_source, batch_share_per_px: int | None = None, max_chain: int = 4):
        import torch
        self.torch = torch
        self.ctxs = ctx
        self.src = frame_source          # (spec, t) -> device frame tuple
        # batch-pool bytes per admitted pixel: by default what a full chain of the stream
        # takes in a batch (max_chain groups and their frames, nv_batch_bytes_per_px)
        self.share = batch_share_per_px
        self.max_chain = max_chain       # a chain of k frames keeps k + 1 frames resident
        self._pool = {}
        self._ctx_of = {}                # id(stream handle) -> its context

    def now(self):
        return time.perf_counter()

    @staticmethod
    def _fmt(spec):
        from . import binding as B
        return B.fmt_struct(spec.width, spec.height, spec.bits, spec.chroma, matrix=spec.matrix, full=spec.full,
                            centre=spec.centre)

    def footprint(self, spec):
        ctx = select_context(self.ctxs, spec)
        if ctx is None:
            return UNSERVABLE
        hp, wp = (spec.height + 7) // 8 * 8, (spec.width + 7) // 8 * 8
        slot = hp * wp * (12 + ctx.channels * (4 if ctx.feat_dtype == torch_float32() else 2))
        share = self.share
        if share is None:
            per_group, per_frame = ctx.batch_bytes_per_px()
            share = self.max_chain * per_group + (self.max_chain + 1) * per_frame
        return ctx.stream_footprint(self._fmt(spec)) + (self.max_chain - 1) * slot + share * hp * wp

    def open(self, spec):
        ctx = select_context(self.ctxs, spec)
        key = (spec.width, spec.height, spec.bits, spec.chroma, spec.matrix, spec.full, spec.centre)
        if self._pool.get(key):
            st = self._pool[key].pop()
            st.reset()
        else:
            st = ctx.open_stream(self._fmt(spec))
            st.pool_key = key
        self._ctx_of[id(st)] = ctx
        return st

    def submit(self, reqs):
        torch = self.torch
        # one batch call per context, outputs returned in request order
        by_ctx = {}
        for k, (st, spec, idx, end) in enumerate(reqs):
            ctx = self._ctx_of[id(st)]
            by_ctx.setdefault(id(ctx), (ctx, []))[1].append(k)
        outs = [None] * len(reqs)
        for ctx, ks in by_ctx.values():
            batch = [(reqs[k][0], [self.src(reqs[k][1], t) for t in reqs[k][2]], None, reqs[k][3]) for k in ks]
            for k, o in zip(ks, ctx.enhance_batch(batch)):
                outs[k] = o
        ev = torch.cuda.Event()
        ev.record()
        return {"event": ev, "outs": outs}

    def poll(self, ticket):
        return ticket["event"].query()

    def wait_any(self, tickets, timeout):
        t_end = time.perf_counter() + timeout
        while time.perf_counter() < t_end:
            if any(t["event"].query() for t in tickets):
                return
            time.sleep(0.0002)

    def outputs(self, ticket):
        return ticket["outs"]

    def release(self, ticket):
        ticket["outs"] = None

    def close(self, st):
        self._pool.setdefault(st.pool_key, []).append(st)

    def shutdown(self):
        for lst in self._pool.values():
            for st in lst:
                st.close()
        self._pool = {}
