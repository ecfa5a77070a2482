"""Host-side scheduling rules of the serving loop, with an executor that never touches a
device (so it runs on the CPU): admission by footprint, frame order, batch limits, one
record per group, completion only after submission."""
import itertools

import pytest

from paper_2308_03121_amd.serving import Server, StreamSpec, poisson_workload


class FakeExecutor:
    def __init__(self, bytes_per_px=10, polls_to_finish=2):
        self.t = 0.0
        self.bytes_per_px = bytes_per_px
        self.polls = polls_to_finish
        self.open_streams = set()
        self.max_open = 0
        self.submitted = []          # list of requests per batch
        self.pushed = {}             # sid -> frames pushed so far
        self.ids = itertools.count()

    def now(self):
        self.t += 0.001              # time advances by 1 ms per look at the clock
        return self.t

    def footprint(self, spec):
        return spec.width * spec.height * self.bytes_per_px

    def open(self, spec):
        h = (spec.sid, next(self.ids))
        self.open_streams.add(h)
        self.max_open = max(self.max_open, len(self.open_streams))
        self.pushed[spec.sid] = 0
        return h

    def submit(self, reqs):
        for h, spec, idx, end in reqs:
            assert h in self.open_streams
            assert idx == list(range(self.pushed[spec.sid], self.pushed[spec.sid] + len(idx)))
            self.pushed[spec.sid] += len(idx)
            if end:
                assert self.pushed[spec.sid] == spec.n_frames
        self.submitted.append(reqs)
        return {"left": self.polls}

    def poll(self, ticket):
        ticket["left"] -= 1
        return ticket["left"] <= 0

    def wait_any(self, tickets, timeout):
        pass

    def outputs(self, ticket):
        return None

    def release(self, ticket):
        pass

    def close(self, h):
        self.open_streams.remove(h)


def _specs(n=6, frames=12, gap=0.004):
    return [StreamSpec(i, 64 + 16 * (i % 2), 48, 8, 420, [0.003 * i + gap * k for k in range(frames)])
            for i in range(n)]


def test_every_group_recorded_once_and_completed():
    ex = FakeExecutor()
    srv = Server(ex, hbm_budget=10 ** 9)
    specs = _specs()
    rep = srv.run(specs, time_scale=1.0)
    assert rep["groups"] == sum(s.n_frames for s in specs)
    for s in specs:
        recs = sorted((r for r in srv.records if r.sid == s.sid), key=lambda r: r.index)
        assert [r.index for r in recs] == list(range(s.n_frames))
        for r in recs:
            assert r.done >= r.ready
    assert not ex.open_streams


def test_admission_respects_budget():
    ex = FakeExecutor(bytes_per_px=10)
    one = 80 * 48 * 10
    srv = Server(ex, hbm_budget=2 * one)
    specs = _specs(n=6)
    rep = srv.run(specs)
    assert ex.max_open <= 2
    assert srv.rejected == 0 and len(srv.admissions) == 6
    # the streams beyond the first two waited for budget, and the report says so
    assert rep["admission_waited"] >= 4 and rep["admission_wait_max_ms"] > 0.0
    ex2 = FakeExecutor(bytes_per_px=10)
    rep2 = Server(ex2, hbm_budget=10 ** 9).run(_specs(n=6))
    # (the fake clock advances 1 ms per look, so even immediate admissions read a few ms)
    assert rep2["admission_wait_max_ms"] < 10.0 < rep["admission_wait_max_ms"]


def test_too_large_stream_is_rejected():
    ex = FakeExecutor(bytes_per_px=10)
    srv = Server(ex, hbm_budget=64 * 48 * 10)
    specs = _specs(n=2)            # stream 1 is 80 px wide: over budget on its own
    rep = srv.run(specs)
    assert rep["rejected"] == 1 and rep["admitted"] == 1


def test_batch_limits():
    ex = FakeExecutor(polls_to_finish=50)
    srv = Server(ex, hbm_budget=10 ** 9, max_frames=5, max_chain=2)
    srv.run(_specs(n=4, frames=10, gap=0.0005))
    for reqs in ex.submitted:
        assert sum(len(idx) for _h, _s, idx, _e in reqs) <= 5
        assert all(len(idx) <= 2 for _h, _s, idx, _e in reqs)


def test_poisson_workload_shape():
    specs = poisson_workload(n_streams=16, rate_total=40.0, seed=3)
    assert len(specs) == 16
    assert {(s.width, s.height) for s in specs} <= {(960, 540), (1920, 1080)}
    assert all(30 <= s.n_frames <= 300 for s in specs)
    for s in specs:
        assert all(b > a for a, b in zip(s.arrivals, s.arrivals[1:]))
        gaps = [b - a for a, b in zip([0] + s.scene_starts, s.scene_starts)]
        assert all(10 <= g <= 60 for g in gaps)
    rate = sum(s.n_frames for s in specs) / sum(s.arrivals[-1] - s.arrivals[0] for s in specs) * 16
    assert 20 < rate < 80


def test_network_selected_by_stream_colourspace():
    """Each stream is served by the network trained for its colourspace (matrix, range);
    a stream whose colourspace has no network cannot be admitted under any budget."""
    from paper_2308_03121_amd.serving import UNSERVABLE, select_context

    class Ctx:
        def __init__(self, matrix, full):
            self.colourspace = (matrix, full)

    c709, c601f = Ctx(709, False), Ctx(601, True)
    ctxs = {c709.colourspace: c709, c601f.colourspace: c601f}
    mk = lambda m, f, c=False: StreamSpec(0, 64, 32, 8, 420, [0.0], matrix=m, full=f, centre=c)  # noqa: E731
    assert select_context(ctxs, mk(709, False)) is c709
    assert select_context(ctxs, mk(601, True, True)) is c601f     # siting does not select a network
    assert select_context(ctxs, mk(2020, False)) is None
    assert select_context(c709, mk(709, False)) is c709 and select_context(c709, mk(601, False)) is None

    class Exec(FakeExecutor):
        def footprint(self, spec):
            return UNSERVABLE if select_context(ctxs, spec) is None else super().footprint(spec)

    ex = Exec()
    specs = [StreamSpec(0, 64, 32, 8, 420, [0.0, 0.01], matrix=709), StreamSpec(1, 64, 32, 8, 420, [0.0], matrix=2020),
             StreamSpec(2, 64, 32, 8, 420, [0.0, 0.02], matrix=601, full=True)]
    srv = Server(ex, hbm_budget=1 << 40)
    rep = srv.run(specs)
    assert rep["rejected"] == 1 and rep["admitted"] == 2
    assert rep["groups"] == 4
