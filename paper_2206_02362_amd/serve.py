"""Request loop: modeling, extended Born and gradient requests on one GPU.

Requests on grids of different sizes arrive at any time.  The server owns a
fixed number of slots; a slot is a HIP stream plus its own library context
(the library runs one stream per context).  Velocity models are registered
once and stay resident on the device; a request names one.  Admission is
first come, first served by default: the head of the queue starts as soon as
a slot is free and its device footprint (fwime_footprint for its operator,
shot count and grid, plus its outputs) fits in what the running requests
leave of the HBM budget, and, while others run, its stencil workgroups
(56 x 32 tiles of every shot) fit beside theirs under a fill bound.  A
request big enough to fill the GPU alone therefore runs alone, as in
one-at-a-time order, while small requests, which leave most compute units
idle, overlap: a request that arrives while others run starts on a free slot
and its kernels run beside theirs.  With policy="short_first" the request of
least work (cell-updates) among those that can start goes first, unless the
head has waited longer than an aging bound.

Modeling requests are batched continuously (engine=True): they go to one
fwime_engine, whose time loop runs in rounds of a fixed number of time steps
on its own stream; a request admitted while the loop runs joins it at the
next round boundary and shares every launch with the jobs already in it (each
at its own time index), and leaves it when its last sample is recorded.  The
server keeps at most two rounds in flight, so new jobs wait at most about a
round.  With engine=False, modeling requests that wait back to back at the
head of the queue are merged into one fwime_model_batch call instead.
Completion is observed with events.  Each context keeps its scratch arena
(checkpoints, wavefield rings, tables) between requests, so a slot reuses
device memory instead of reallocating it; idle slots give their arenas back
(fwime_ctx_trim) when the arenas held by all slots exceed the budget.

Every numerical step runs in the HIP library; this module only schedules.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass
from typing import Any, Callable

import numpy as np
import torch

from ._abi import (FWIME_OP_BORN_ADJ, FWIME_OP_BORN_FWD, FWIME_OP_GRADIENT, FWIME_OP_MODEL, Context, Engine,
                   Geometry, Grid, footprint)

_OPS = {"model": FWIME_OP_MODEL, "born_fwd": FWIME_OP_BORN_FWD, "born_adj": FWIME_OP_BORN_ADJ,
        "gradient": FWIME_OP_GRADIENT}
# wavefield propagations per shot: modeling 1; Born forward and adjoint 2
# (background + scattered / adjoint); gradient 6 (background and Born
# forward, the adjoint and its Born-type partner, and the two recomputation
# passes over the checkpoints)
PROPAGATIONS = {"model": 1, "born_fwd": 2, "born_adj": 2, "gradient": 6}


@dataclass
class Request:
    kind: str                            # model | born_fwd | born_adj | gradient
    model: Any                           # key of a registered velocity model
    geom: Geometry
    nt: int
    nh: int = 1                          # subsurface offsets (Born, gradient)
    ptilde: torch.Tensor | None = None   # [nh][nx][nz]: born_fwd, gradient
    data: torch.Tensor | None = None     # [nshots][nrec][nt]: born_adj input
    dobs: torch.Tensor | None = None     # [nshots][nrec][nt]: gradient
    eps: float = 0.0
    dso: np.ndarray | None = None        # [nh] DSO weights: gradient
    tag: Any = None
    # filled in by the server
    id: int = -1
    grid: Grid | None = None
    t_arrival: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    slot: int = -1
    result: Any = None
    error: Exception | None = None
    reserved: int = 0
    tiles_held: int = 0
    merged: int = 1                      # requests sharing this one's launch
    ticket: int = -1                     # engine job (continuously batched modeling)
    _ready: Any = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival

    def cell_updates(self) -> float:
        g = self.grid
        return PROPAGATIONS[self.kind] * self.geom.nshots * (g.nz + 2 * g.nb) * (g.nx + 2 * g.nb) * (g.nt - 1)

    def tiles(self) -> int:
        """Workgroups of one stencil launch over all its shots (56 x 32 cell tiles)."""
        g = self.grid
        return self.geom.nshots * (-(-(g.nz + 2 * g.nb) // 56)) * (-(-(g.nx + 2 * g.nb) // 32))


def request_bytes(req: Request) -> int:
    """Device bytes a request holds while it runs: library scratch + outputs."""
    g = req.grid
    nh = req.nh if req.kind != "model" else 1
    b = footprint(g, req.geom.nshots, req.geom.nrec, nh, _OPS[req.kind])
    out = 4 * req.geom.nshots * req.geom.nrec * g.nt if req.kind in ("model", "born_fwd") else 0
    if req.kind in ("born_adj", "gradient"):
        out += 4 * (nh + 1) * g.nx * g.nz + 8
    return b + out


class _Slot:
    def __init__(self, device: int, budget: int):
        self.stream = torch.cuda.Stream(device)
        self.ctx = Context(device, budget)
        self.reqs: list[Request] = []
        self.event = None

    def held_bytes(self) -> int:
        return self.ctx.info()["arena_bytes"]

    def trim(self):
        self.ctx.trim(self.stream.cuda_stream)

    def close(self):
        self.stream.synchronize()
        self.ctx.close()


class _EngineLane:
    """The continuous-batching engine with its own stream and context, a
    stream for checking newly admitted inputs, and the rounds in flight."""

    def __init__(self, device: int, budget: int, steps: int, max_jobs: int = 512):
        self.stream = torch.cuda.Stream(device)
        self.check_stream = torch.cuda.Stream(device)
        self.ctx = Context(device, budget)
        self.engine = Engine(self.ctx, self.stream, steps, max_jobs)
        self.inflight: collections.deque = collections.deque()
        self.reqs: dict[int, Request] = {}

    def submit(self, r: Request, vel: torch.Tensor) -> None:
        with torch.cuda.stream(self.stream):
            r.result = torch.empty((r.geom.nshots, r.geom.nrec, r.grid.nt), device=vel.device,
                                   dtype=torch.float32)
        self.check_stream.wait_event(r._ready)
        r.ticket = self.engine.submit(r.grid, vel, r.geom, r.result, self.check_stream)
        self.reqs[r.ticket] = r

    def pump(self) -> None:
        """Keep two rounds in flight while jobs remain."""
        while self.inflight and self.inflight[0].query():
            self.inflight.popleft()
        while len(self.inflight) < 2:
            inf = self.engine.info()
            if inf["pending"] == 0 and inf["active"] == 0:
                return
            self.engine.run()
            ev = torch.cuda.Event()
            ev.record(self.stream)
            self.inflight.append(ev)

    def finished(self) -> list[Request]:
        return [self.reqs.pop(t) for t in self.engine.poll()]

    def busy(self) -> bool:
        return bool(self.reqs)

    def close(self):
        self.engine.close()
        self.stream.synchronize()
        self.ctx.close()


class Server:
    """FIFO admission by HBM footprint onto `slots` concurrent streams, with
    modeling requests continuously batched in one engine (engine=True).

    hbm_budget: bytes the running requests may hold together (default 80 % of
    the free device memory when the server starts).  merge_models: the most
    modeling requests one batched call may serve when there is no engine (1
    turns merging off).  engine_steps: time steps per engine round.
    policy: "fcfs" (arrival order; nothing overtakes the head) or
    "short_first" (the least work among the requests that can start now; a
    head that has waited aging_s seconds goes first).
    fill_tiles: while requests run, another starts only if the stencil
    workgroups of all of them stay within this bound (None: no bound).  The
    default, 4096, is about three waves of two-step stencil workgroups over
    the 256 compute units, beyond which a launch keeps the GPU busy alone.
    """

    def __init__(self, device: int = 0, slots: int = 3, hbm_budget: int | None = None, merge_models: int = 8,
                 engine: bool = False, engine_steps: int = 64, policy: str = "fcfs", aging_s: float = 30.0,
                 fill_tiles: int | None = 4096,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep):
        if policy not in ("fcfs", "short_first"):
            raise ValueError("policy must be 'fcfs' or 'short_first'")
        self.policy = policy
        self.aging_s = float(aging_s)
        self.fill_tiles = None if fill_tiles is None else int(fill_tiles)
        self.running_tiles = 0
        self.device = device
        self.clock = clock
        self.sleep = sleep
        if hbm_budget is None:
            hbm_budget = self._default_budget(device)
        self.budget = int(hbm_budget)
        self.merge_models = max(1, int(merge_models))
        self.models: dict[Any, tuple[Grid, torch.Tensor]] = {}
        self.slots = [self._new_slot(k) for k in range(slots)]
        self.lane = self._new_engine(engine_steps) if engine else None
        self.queue: collections.deque[Request] = collections.deque()
        self.done: list[Request] = []
        self.reserved = 0
        self.peak_reserved = 0
        self.admit_order: list[int] = []
        self._next_id = 0

    # -- hooks a host-only test replaces ---------------------------------------
    def _default_budget(self, device) -> int:
        free, _ = torch.cuda.mem_get_info(device)
        return int(0.8 * free)

    def _new_slot(self, k: int):
        return _Slot(self.device, self.budget)

    def _new_engine(self, steps: int):
        return _EngineLane(self.device, self.budget, steps)

    def _need(self, req: Request) -> int:
        return request_bytes(req)

    def _finished(self, slot) -> bool:
        return slot.event.query()

    # -- resident models --------------------------------------------------------
    def add_model(self, key, grid: Grid, vel: torch.Tensor) -> None:
        """Keep a velocity model [nx][nz] resident; requests name it by key.

        grid gives the model's nz, nx, sponge, spacing and dt; each request
        supplies its own nt."""
        self.models[key] = (grid, vel)

    def grid_for(self, req: Request) -> Grid:
        g, _ = self.models[req.model]
        return Grid(g.nz, g.nx, g.nb, req.nt, g.dz, g.dx, g.dt, g.sponge_alpha, g.free_surface)

    # -- public -----------------------------------------------------------------
    def submit(self, req: Request, t_arrival: float | None = None) -> Request:
        if req.model not in self.models:
            raise KeyError(f"model {req.model!r} is not registered")
        req.id = self._next_id
        self._next_id += 1
        req.grid = self.grid_for(req)
        req.t_arrival = self.clock() if t_arrival is None else t_arrival
        req._ready = self._mark_inputs_ready()
        self.queue.append(req)
        return req

    def close(self) -> None:
        """Wait for the slots' and the engine's work and release their contexts."""
        for s in self.slots:
            s.close()
        if self.lane is not None:
            self.lane.close()

    def busy(self) -> bool:
        return (bool(self.queue) or any(s.reqs for s in self.slots)
                or (self.lane is not None and self.lane.busy()))

    def poll(self) -> None:
        self._retire()
        self._admit()
        if self.lane is not None:
            self.lane.pump()

    def drain(self) -> list[Request]:
        while self.busy():
            self.poll()
            self.sleep(1e-4)
        return self.done

    def replay(self, requests: list[Request], arrivals: list[float]) -> list[Request]:
        """Submit each request at its arrival offset (s, ascending), run all to completion."""
        start = self.clock()
        i, n = 0, len(requests)
        while i < n or self.busy():
            now = self.clock() - start
            while i < n and arrivals[i] <= now:
                self.submit(requests[i], start + arrivals[i])
                i += 1
            self.poll()
            if i < n or self.busy():
                self.sleep(1e-4)
        return self.done

    @staticmethod
    def stats(done: list[Request]) -> dict:
        lat = np.array([r.latency for r in done], dtype=np.float64)
        t0 = min(r.t_arrival for r in done)
        t1 = max(r.t_done for r in done)
        cells = sum(r.cell_updates() for r in done)
        return {"requests": len(done), "p50_s": float(np.percentile(lat, 50)),
                "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
                "makespan_s": float(t1 - t0), "requests_per_s": len(done) / (t1 - t0),
                "cell_updates_per_s": cells / (t1 - t0),
                "errors": sum(r.error is not None for r in done)}

    # -- internals --------------------------------------------------------------
    def _mark_inputs_ready(self):
        # the request's tensors were written on the caller's stream: slot
        # streams wait for this event before reading them
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(self.device))
        return ev

    def _retire(self):
        for s in self.slots:
            if s.reqs and self._finished(s):
                t = self.clock()
                for r in s.reqs:
                    r.t_done = t
                    self.reserved -= r.reserved
                    self.running_tiles -= r.tiles_held
                    self.done.append(r)
                s.reqs = []
                s.event = None
        if self.lane is not None:
            fin = self.lane.finished()
            t = self.clock()
            for r in fin:
                r.t_done = t
                self.reserved -= r.reserved
                self.running_tiles -= r.tiles_held
                self.done.append(r)
        held = sum(s.held_bytes() for s in self.slots)
        if held > self.budget:
            for s in self.slots:
                if not s.reqs and held > self.budget:
                    h = s.held_bytes()
                    s.trim()
                    held -= h

    def _pick(self):
        """Index in the queue of the next request to start, or None.

        fcfs: the head, once a slot (unless it goes to the engine), its
        memory and, beside running requests, its share of the compute units
        are free; nothing overtakes it.  short_first: the request of the
        least work (cell-updates) among those that can start now, except
        that a head that has waited longer than `aging_s` goes first and
        holds back the others until it starts."""
        running = any(s.reqs for s in self.slots) or (self.lane is not None and self.lane.busy())
        free_slot = any(not s.reqs for s in self.slots)

        def startable(r):
            if not (self.lane is not None and r.kind == "model") and not free_slot:
                return False
            if not running:
                return True
            if self.fill_tiles is not None and self.running_tiles + r.tiles() > self.fill_tiles:
                return False
            return self.reserved + min(self._need(r), self.budget) <= self.budget

        if self.policy == "fcfs" or self.clock() - self.queue[0].t_arrival > self.aging_s:
            return 0 if startable(self.queue[0]) else None
        order = sorted(range(len(self.queue)), key=lambda i: (self.queue[i].cell_updates(), i))
        return next((i for i in order if startable(self.queue[i])), None)

    def _admit(self):
        while self.queue:
            i = self._pick()
            if i is None:
                return
            head = self.queue[i]
            del self.queue[i]
            need = min(self._need(head), self.budget)
            if self.lane is not None and head.kind == "model":
                head.reserved = need
                head.tiles_held = head.tiles()
                self.reserved += need
                self.running_tiles += head.tiles_held
                self.peak_reserved = max(self.peak_reserved, self.reserved)
                head.t_admit = self.clock()
                self.admit_order.append(head.id)
                try:
                    self._engine_submit(head)
                except Exception as e:      # reported on the request; the server keeps going
                    head.error = e
                    head.t_done = self.clock()
                    self.reserved -= need
                    self.running_tiles -= head.tiles_held
                    self.done.append(head)
                continue
            k = next(k for k, s in enumerate(self.slots) if not s.reqs)
            group = [head]
            head.reserved = need
            total = need
            if head.kind == "model" and i == 0:
                while (self.queue and self.queue[0].kind == "model" and len(group) < self.merge_models):
                    nxt = self.queue[0]
                    nn = min(self._need(nxt), self.budget)
                    if self.reserved + total + nn > self.budget:
                        break
                    nxt.reserved = nn
                    total += nn
                    group.append(self.queue.popleft())
            self.reserved += total
            self.peak_reserved = max(self.peak_reserved, self.reserved)
            now = self.clock()
            for r in group:
                r.tiles_held = r.tiles()
                self.running_tiles += r.tiles_held
                r.slot = k
                r.t_admit = now
                r.merged = len(group)
                self.admit_order.append(r.id)
            self._start(self.slots[k], group)

    def _engine_submit(self, r: Request):
        _, vel = self.models[r.model]
        self.lane.submit(r, vel)

    def _start(self, s: _Slot, group: list[Request]):
        s.reqs = group
        try:
            with torch.cuda.stream(s.stream):
                for r in group:
                    s.stream.wait_event(r._ready)
                self._run(s.ctx, group)
        except Exception as e:         # reported on the request; the server keeps going
            for r in group:
                r.error = e
        s.event = torch.cuda.Event()
        s.event.record(s.stream)

    def _run(self, ctx: Context, group: list[Request]):
        if len(group) > 1:             # merged modeling requests
            jobs = []
            for r in group:
                _, vel = self.models[r.model]
                jobs.append((r.grid, vel, r.geom))
            for r, out in zip(group, ctx.model_batch(jobs)):
                r.result = out
            return
        r = group[0]
        _, vel = self.models[r.model]
        if r.kind == "model":
            r.result = ctx.model(r.grid, vel, r.geom)
        elif r.kind == "born_fwd":
            r.result = ctx.born_ext_fwd(r.grid, vel, r.geom, r.ptilde)
        elif r.kind == "born_adj":
            r.result = ctx.born_ext_adj(r.grid, vel, r.geom, r.data, r.nh)
        elif r.kind == "gradient":
            dso = r.dso if r.dso is not None else np.ones(r.nh)
            r.result = ctx.gradient(r.grid, vel, r.geom, r.ptilde, r.dobs, r.eps, dso)
        else:
            raise ValueError(f"unknown request kind {r.kind!r}")
