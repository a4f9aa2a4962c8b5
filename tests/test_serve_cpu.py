"""Host-side scheduling of the request loop (no GPU).

The server's slot, footprint and completion hooks are replaced by a fake
device with a virtual clock: each request runs for a stated time and holds a
stated number of bytes.  Checked: admission never holds more than the HBM
budget, requests start in arrival order, a seeded Poisson replay is
deterministic, an oversized request runs alone, a request whose stencil
workgroups would overfill the GPU beside running ones waits, modeling
requests at the head of the queue merge, idle arenas are trimmed under memory pressure, and
the latency percentiles.
"""
import numpy as np
import pytest
import torch

from paper_2206_02362_amd import Geometry, Grid
from paper_2206_02362_amd.serve import Request, Server


class FakeSlot:
    def __init__(self):
        self.reqs = []
        self.finish = 0.0
        self.held = 0
        self.trims = 0

    def held_bytes(self):
        return self.held

    def trim(self):
        self.held = 0
        self.trims += 1


class FakeLane:
    """Continuous-batching engine on the virtual clock: a job joins at once
    and runs r.tag['dur'] seconds beside the others."""

    def __init__(self, srv):
        self.srv = srv
        self.reqs = {}
        self.joined = []

    def submit(self, r, vel):
        r.ticket = len(self.joined)
        self.joined.append((r.ticket, self.srv.t))
        self.reqs[r.ticket] = (r, self.srv.t + r.tag["dur"])

    def pump(self):
        pass

    def finished(self):
        out = [t for t, (r, f) in self.reqs.items() if self.srv.t >= f]
        return [self.reqs.pop(t)[0] for t in out]

    def busy(self):
        return bool(self.reqs)


class FakeServer(Server):
    """Virtual clock; request r runs r.tag['dur'] seconds and needs r.tag['bytes']."""

    def __init__(self, **kw):
        self.t = 0.0
        self.concurrent = []
        super().__init__(clock=lambda: self.t, sleep=self._advance, **kw)
        self.add_model("m", Grid(20, 30, 4, 100, 10.0, 10.0, 1e-3), None)

    def _advance(self, dt):
        self.t += 1e-3

    def _new_slot(self, k):
        return FakeSlot()

    def _new_engine(self, steps):
        return FakeLane(self)

    def _need(self, r):
        return r.tag["bytes"]

    def _finished(self, s):
        return self.t >= s.finish

    def _mark_inputs_ready(self):
        return None

    def _start(self, s, group):
        s.reqs = group
        s.finish = self.t + max(r.tag["dur"] for r in group)
        s.held = max(s.held, sum(r.reserved for r in group))
        self.concurrent.append(sum(r.reserved for sl in self.slots for r in sl.reqs))


def _geom(ns=1):
    return Geometry(np.full(ns, 2), np.arange(ns), np.full((ns, 3), 2), np.tile(np.arange(3), (ns, 1)),
                    torch.zeros(ns, 100))


def _req(kind, nbytes, dur):
    return Request(kind, "m", _geom(), 100, tag={"bytes": nbytes, "dur": dur})


def _poisson(seed, n, budget, rate=20.0):
    rng = np.random.default_rng(seed)
    arrivals = list(np.cumsum(rng.exponential(1.0 / rate, n)))
    kinds = ["model", "born_fwd", "born_adj", "gradient"]
    reqs = [_req(kinds[int(rng.integers(4))], int(rng.uniform(0.05, 0.7) * budget), float(rng.uniform(0.05, 0.5)))
            for _ in range(n)]
    return reqs, arrivals


def test_admission_never_exceeds_budget_and_is_fifo():
    budget = 1000
    srv = FakeServer(slots=4, hbm_budget=budget)
    reqs, arr = _poisson(1, 60, budget)
    done = srv.replay(reqs, arr)
    assert len(done) == 60 and all(r.error is None for r in done)
    assert srv.peak_reserved <= budget
    assert max(srv.concurrent) <= budget
    assert srv.reserved == 0
    assert srv.admit_order == sorted(srv.admit_order)
    # requests did overlap: some started while another was still running
    assert any(r.t_admit < q.t_done and q.t_admit < r.t_admit for r in done for q in done if q is not r)


def test_overlap_happens_when_memory_allows():
    srv = FakeServer(slots=3, hbm_budget=1000)
    reqs = [_req("born_fwd", 300, 1.0) for _ in range(3)]
    done = srv.replay(reqs, [0.0, 0.0, 0.0])
    # all three fit together: they start at once and finish after ~1 s
    assert max(r.t_admit for r in done) < 0.01
    assert max(r.latency for r in done) < 1.01


def test_waits_for_memory_in_arrival_order():
    srv = FakeServer(slots=3, hbm_budget=1000)
    a = _req("gradient", 800, 1.0)
    b = _req("born_adj", 500, 0.2)     # does not fit beside a
    c = _req("model", 100, 0.2)        # would fit, but must not overtake b
    done = srv.replay([a, b, c], [0.0, 0.001, 0.002])
    t = {r.id: r for r in done}
    assert t[1].t_admit >= t[0].t_done - 1e-9
    assert t[2].t_admit >= t[1].t_admit
    assert srv.admit_order == [0, 1, 2]


def test_oversized_request_runs_alone():
    srv = FakeServer(slots=3, hbm_budget=1000)
    small = _req("model", 100, 0.5)
    big = _req("gradient", 5000, 0.5)
    done = srv.replay([small, big], [0.0, 0.01])
    t = {r.id: r for r in done}
    assert t[1].reserved == 1000              # capped at the budget
    assert t[1].t_admit >= t[0].t_done - 1e-9
    assert srv.peak_reserved <= 1000


def test_replay_is_deterministic():
    out = []
    for _ in range(2):
        srv = FakeServer(slots=3, hbm_budget=1000)
        reqs, arr = _poisson(7, 40, 1000)
        done = srv.replay(reqs, arr)
        out.append([(r.id, round(r.t_admit, 9), round(r.t_done, 9), r.slot) for r in sorted(done, key=lambda r: r.id)])
    assert out[0] == out[1]


def test_head_model_requests_merge():
    srv = FakeServer(slots=1, hbm_budget=1000, merge_models=8)
    blocker = _req("gradient", 200, 0.5)
    models = [_req("model", 100, 0.3) for _ in range(3)]
    tail = _req("born_fwd", 100, 0.1)
    done = srv.replay([blocker] + models + [tail], [0.0, 0.01, 0.02, 0.03, 0.04])
    t = {r.id: r for r in done}
    assert [t[i].merged for i in (1, 2, 3)] == [3, 3, 3]
    assert len({t[i].t_admit for i in (1, 2, 3)}) == 1
    assert t[4].merged == 1 and t[4].t_admit > t[1].t_admit

    srv = FakeServer(slots=1, hbm_budget=1000, merge_models=1)
    done = srv.replay([blocker] + models + [tail], [0.0, 0.01, 0.02, 0.03, 0.04])
    assert all(r.merged == 1 for r in done)


def test_merge_respects_budget():
    srv = FakeServer(slots=1, hbm_budget=1000, merge_models=8)
    reqs = [_req("model", 400, 0.1) for _ in range(4)]
    done = srv.replay(reqs, [0.0] * 4)
    assert [r.merged for r in sorted(done, key=lambda r: r.id)] == [2, 2, 2, 2]
    assert srv.peak_reserved <= 1000


def test_engine_takes_modeling_requests_as_they_arrive():
    # modeling requests join the engine at once, beside one another and beside
    # slot work, without waiting for a free slot; arrival order and the
    # budget still hold
    srv = FakeServer(slots=1, hbm_budget=1000, engine=True)
    blocker = _req("gradient", 300, 1.0)
    models = [_req("model", 100, 0.3) for _ in range(4)]
    done = srv.replay([blocker] + models, [0.0, 0.1, 0.2, 0.25, 0.3])
    t = {r.id: r for r in done}
    for i in range(1, 5):
        assert t[i].t_admit == pytest.approx(t[i].t_arrival, abs=2e-3)   # no wait for the busy slot
        assert t[i].t_done < t[0].t_done
    assert len(srv.lane.joined) == 4 and srv.admit_order == [0, 1, 2, 3, 4]
    assert srv.peak_reserved <= 1000 and srv.reserved == 0


def test_engine_respects_budget_and_arrival_order():
    srv = FakeServer(slots=2, hbm_budget=1000, engine=True)
    a = _req("model", 700, 0.5)
    b = _req("model", 500, 0.2)         # does not fit beside a: waits
    c = _req("born_fwd", 100, 0.1)      # would fit, but must not overtake b
    done = srv.replay([a, b, c], [0.0, 0.01, 0.02])
    t = {r.id: r for r in done}
    assert t[1].t_admit >= t[0].t_done - 1e-9
    assert t[2].t_admit >= t[1].t_admit
    assert srv.peak_reserved <= 1000
    reqs, arr = _poisson(3, 60, 1000)
    srv = FakeServer(slots=3, hbm_budget=1000, engine=True)
    done = srv.replay(reqs, arr)
    assert len(done) == 60 and srv.reserved == 0 and srv.peak_reserved <= 1000
    assert srv.admit_order == sorted(srv.admit_order)


def _sized(kind, nbytes, dur, nshots):
    r = _req(kind, nbytes, dur)
    r.geom = _geom(nshots)
    return r


def test_short_first_lets_small_requests_by_and_ages():
    # one slot busy with a long gradient; a big and a small Born request
    # wait: short_first starts the small one first, fcfs keeps arrival order
    for policy, first in (("short_first", 2), ("fcfs", 1)):
        srv = FakeServer(slots=1, hbm_budget=1000, policy=policy, aging_s=100.0)
        reqs = [_sized("gradient", 100, 1.0, 1), _sized("born_fwd", 100, 0.5, 8), _sized("born_fwd", 100, 0.1, 1)]
        done = srv.replay(reqs, [0.0, 0.01, 0.02])
        t = {r.id: r for r in done}
        assert srv.admit_order[:2] == [0, first]
        assert t[first].t_admit == pytest.approx(t[0].t_done, abs=2e-3)
    # a head that waited past the aging bound goes first
    srv = FakeServer(slots=1, hbm_budget=1000, policy="short_first", aging_s=0.5)
    reqs = [_sized("gradient", 100, 1.0, 1), _sized("born_fwd", 100, 0.5, 8), _sized("born_fwd", 100, 0.1, 1)]
    srv.replay(reqs, [0.0, 0.01, 0.02])
    assert srv.admit_order == [0, 1, 2]
    # budget and completion still hold on a Poisson stream
    reqs, arr = _poisson(5, 60, 1000)
    srv = FakeServer(slots=3, hbm_budget=1000, engine=True, policy="short_first")
    done = srv.replay(reqs, arr)
    assert len(done) == 60 and srv.reserved == 0 and srv.peak_reserved <= 1000
    with pytest.raises(ValueError):
        FakeServer(policy="lifo")


def test_fill_bound_runs_gpu_filling_requests_alone():
    # the fake grid has 2 stencil tiles per shot; fill bound 10 tiles
    def reqs():
        return [_sized("gradient", 100, 1.0, 4),     # 8 tiles
                _sized("born_fwd", 100, 0.2, 2),     # 4 tiles: 12 > 10 beside the first, waits
                _sized("model", 100, 0.2, 1),        # 2 tiles: would fit beside the first
                _sized("born_adj", 100, 0.3, 6)]     # 12 tiles: fills the GPU alone
    arr = [0.0, 0.01, 0.02, 0.03]
    srv = FakeServer(slots=3, hbm_budget=1000, fill_tiles=10)
    t = {r.id: r for r in srv.replay(reqs(), arr)}
    assert [t[i].tiles() for i in range(4)] == [8, 4, 2, 12]
    assert t[1].t_admit >= t[0].t_done - 1e-9           # b waits for a
    assert t[2].t_admit >= t[1].t_admit                 # fcfs: c stays behind b
    assert t[2].t_admit < t[1].t_done                   # then b and c overlap (6 tiles)
    assert t[3].t_admit >= max(t[i].t_done for i in range(3)) - 1e-9   # the big one runs alone
    assert srv.running_tiles == 0 and srv.admit_order == [0, 1, 2, 3]
    # short_first: c starts beside a at once; b still waits for the tiles
    srv = FakeServer(slots=3, hbm_budget=1000, fill_tiles=10, policy="short_first", aging_s=100.0)
    t = {r.id: r for r in srv.replay(reqs(), arr)}
    assert t[2].t_admit == pytest.approx(0.02, abs=2e-3)
    assert t[1].t_admit >= t[0].t_done - 1e-9
    assert srv.admit_order == [0, 2, 1, 3]
    # no bound: b overlaps a
    srv = FakeServer(slots=3, hbm_budget=1000, fill_tiles=None)
    t = {r.id: r for r in srv.replay(reqs(), arr)}
    assert t[1].t_admit < t[0].t_done
    # the engine's modeling jobs count as well
    srv = FakeServer(slots=3, hbm_budget=1000, fill_tiles=10, engine=True)
    t = {r.id: r for r in srv.replay([_sized("model", 100, 1.0, 4), _sized("model", 100, 0.2, 2)], [0.0, 0.01])}
    assert t[1].t_admit >= t[0].t_done - 1e-9 and srv.running_tiles == 0


def test_idle_arenas_trimmed_over_budget():
    srv = FakeServer(slots=2, hbm_budget=1000)
    srv.replay([_req("gradient", 900, 0.1)], [0.0])
    srv.slots[1].held = 900                     # another idle slot still holds its arena
    srv.poll()
    assert sum(s.held for s in srv.slots) <= 1000
    assert sum(s.trims for s in srv.slots) >= 1


def test_unknown_model_rejected():
    srv = FakeServer(slots=1, hbm_budget=1000)
    with pytest.raises(KeyError):
        srv.submit(Request("model", "nope", _geom(), 100, tag={"bytes": 1, "dur": 0.1}))


def test_stats_percentiles():
    rs = []
    for k in range(100):
        r = _req("model", 1, 0.1)
        r.grid = Grid(20, 30, 4, 100, 10.0, 10.0, 1e-3)
        r.t_arrival = 0.0
        r.t_done = float(k + 1)
        rs.append(r)
    st = Server.stats(rs)
    assert st["p50_s"] == pytest.approx(50.5)
    assert st["p99_s"] == pytest.approx(99.01)
    assert st["makespan_s"] == pytest.approx(100.0)
    assert st["cell_updates_per_s"] == pytest.approx(100 * 1 * 28 * 38 * 99 / 100.0)
