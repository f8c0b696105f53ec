"""Request loop that serves DirectL light-field frames from scenes kept resident in device memory.

Each request names a resident scene, a display and a centre-camera pose.  Frames are rendered by plans
(fixed-buffer DirectL frames replayed as HIP graphs, one plan per (scene, display) pair, more than one when the
same pair is in flight twice and memory is spare).  The loop admits requests against a device-memory budget: a
pair's first plan is created when its bytes fit beside the resident scenes and the plans already held, after
evicting idle plans of other pairs in least-recently-used order; a request that cannot get a plan waits (counted
as deferred when it waited for memory) while later requests of other pairs go ahead.  Admitted frames run
concurrently on a few streams; each request's latency runs from its arrival to the completion of its frame, taken
from the frame's GPU completion event (mapped to the host clock through a reference event).  A watchdog reports
frames whose completion has not come by a deadline, and queued requests can be cancelled.

Everything the GPU does goes through the C ABI (`api.Plan`); this module only schedules.
"""

from __future__ import annotations

import dataclasses
import math
import threading
import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field

import numpy as np

from . import api, synth


@dataclass
class Request:
    rid: int
    scene: str
    display: str
    c2w: np.ndarray
    arrival: float  # seconds after the start of the run


@dataclass
class Done:
    rid: int
    scene: str
    display: str
    arrival: float
    launched: float
    finished: float
    deferred: bool
    replans: int
    image: object = None  # the frame, when the server keeps images
    batch: int = 1        # requests in the launch that served it

    @property
    def latency_ms(self) -> float:
        return 1e3 * (self.finished - self.arrival)


def poisson_requests(n: int, rate: float, scenes, displays, seed: int = 2000, distance: float = 3.0) -> list:
    """n requests with exponential inter-arrival times of mean 1/rate; scene, display and orbit angle uniform."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps) - gaps[0]
    si = rng.integers(0, len(scenes), size=n)
    di = rng.integers(0, len(displays), size=n)
    th = rng.uniform(0.0, 2.0 * math.pi, size=n)
    out = []
    for i in range(n):
        eye = (distance * math.sin(th[i]), 0.0, distance * math.cos(th[i]))
        out.append(Request(i, scenes[si[i]], displays[di[i]], synth.look_at_c2w(eye), float(t[i])))
    return out


class Watchdog:
    """Reports work whose completion has not come by a deadline: `arm(key, t)` when it starts, `disarm(key)` when
    it completes, `poll(now)` returns the keys past `deadline_s` that have not been reported yet (each key once).
    Host logic only, driven by the caller's clock."""

    def __init__(self, deadline_s: float):
        self.deadline_s = float(deadline_s)
        self.started: dict = {}
        self.reported: set = set()

    def arm(self, key, t: float) -> None:
        self.started[key] = t
        self.reported.discard(key)

    def disarm(self, key) -> None:
        self.started.pop(key, None)
        self.reported.discard(key)

    def poll(self, now: float) -> list:
        late = [(k, now - t0) for k, t0 in self.started.items()
                if now - t0 > self.deadline_s and k not in self.reported]
        for k, _ in late:
            self.reported.add(k)
        return late


class _PlanEntry:
    def __init__(self, key, plan: api.Plan):
        self.key = key
        self.plan = plan
        self.busy = False
        self.bytes = plan.bytes


class _Slot:
    def __init__(self, torch):
        self.stream = torch.cuda.Stream()
        self.event = torch.cuda.Event(enable_timing=True)
        self.entry = None
        self.reqs = []      # the requests of the launch in flight (one, or a batch of one pair)
        self.launched = 0.0
        self.images = []


@dataclass
class Report:
    done: list
    wall_s: float
    admitted: int
    deferred: int
    waited: int
    replans: int
    plans_created: int
    plans_evicted: int
    hbm_high_water: int
    budget_high_water: int
    budget: int
    resident_bytes: int
    per_display: dict = field(default_factory=dict)
    cancelled: list = field(default_factory=list)   # request ids dropped before launch
    stalled: list = field(default_factory=list)     # (request id, seconds since launch) reported by the watchdog

    def summary(self) -> dict:
        lat = np.array([d.latency_ms for d in self.done]) if self.done else np.zeros(1)
        svc = np.array([1e3 * (d.finished - d.launched) for d in self.done]) if self.done else np.zeros(1)
        out = {
            "requests": len(self.done),
            "frames_per_s": len(self.done) / self.wall_s if self.wall_s > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "service_p50_ms": float(np.percentile(svc, 50)),
            "service_p99_ms": float(np.percentile(svc, 99)),
            "admitted": self.admitted,
            "deferred": self.deferred,
            "waited_for_plan": self.waited,
            "replans": self.replans,
            "plans_created": self.plans_created,
            "plans_evicted": self.plans_evicted,
            # device-wide use (everything on the GPU, incl. memory in use before the server started)
            "hbm_high_water_gb": self.hbm_high_water / 2**30,
            # what the budget bounds: resident scenes + plans
            "budget_high_water_gb": self.budget_high_water / 2**30,
            "budget_gb": self.budget / 2**30,
            "resident_scene_gb": self.resident_bytes / 2**30,
            "cancelled": len(self.cancelled),
            "stalled": len(self.stalled),
            "mean_batch": float(np.mean([d.batch for d in self.done])) if self.done else 0.0,
        }
        per = {}
        for name in sorted({d.display for d in self.done}):
            l = np.array([d.latency_ms for d in self.done if d.display == name])
            v = np.array([1e3 * (d.finished - d.launched) for d in self.done if d.display == name])
            per[name] = {"n": int(l.size), "p50_ms": float(np.percentile(l, 50)), "p99_ms": float(np.percentile(l, 99)),
                         "service_p50_ms": float(np.percentile(v, 50)), "service_p99_ms": float(np.percentile(v, 99))}
        out["per_display"] = per
        return out


class Server:
    """Resident scenes + displays, a plan cache bounded by a device-memory budget, and `n_slots` streams."""

    def __init__(self, ctx: api.Context, budget_bytes: int | None = None, n_slots: int = 4, opts=None,
                 keep_images: bool = False, probe_c2w=None, grow_in_loop: bool = True,
                 watchdog_s: float | None = None, batch_max: int = 1):
        torch = api._torch()
        self.torch = torch
        self.ctx = ctx
        self.opts = opts or api.default_opts()
        self.keep_images = keep_images
        self.probe_c2w = probe_c2w if probe_c2w is not None else synth.look_at_c2w((0.0, 0.0, 3.0))
        self.scenes: dict[str, api.Scene] = {}
        self.scene_bytes: dict[str, int] = {}
        self.displays: dict[str, api.Display] = {}
        self.plans: OrderedDict = OrderedDict()  # id(entry) -> entry, least recently used first
        self.plan_bytes = 0
        self.est: dict = {}  # (scene, display) -> bytes of the last plan made for it
        self.min_keys: dict = {}  # (scene, display) -> capacity a previous overflow asked for
        self.all_chunks: set = set()  # (scene, display) pairs a frame of which needed a later depth chunk
        self.slots = [_Slot(torch) for _ in range(n_slots)]
        free, total = torch.cuda.mem_get_info()
        self.total = total
        self.budget = int(budget_bytes) if budget_bytes is not None else int(0.9 * free)
        self.high_water = total - free
        self.used_high_water = 0
        self.created = self.evicted = 0
        # grow_in_loop: a pair whose plans are all busy may get another plan inside the request loop (from unused
        # budget); otherwise its requests wait for one of its plans (plans made before timing by warm())
        self.grow_in_loop = grow_in_loop
        self.watchdog_s = watchdog_s
        # batch_max > 1: queued requests of the pair that gets a plan are launched with it as one batched launch
        # (dl_plan_render_batch, frames in a row), up to batch_max of them
        self.batch_max = int(batch_max)
        self._cancel_lock = threading.Lock()
        self._cancel: set = set()

    # ---- residency ----
    def add_scene(self, name: str, scene) -> None:
        """Upload a `synth.Scene` (or the 5-tuple of arrays) once; it stays resident."""
        arrays = scene.arrays() if hasattr(scene, "arrays") else scene
        self.scenes[name] = api.Scene(self.ctx, arrays)
        g = self.scenes[name].n
        self.scene_bytes[name] = 59 * 4 * ((g + 63) // 64 * 64)
        self._sample_memory()

    def add_display(self, name: str, display) -> None:
        self.displays[name] = api.Display(self.ctx, display)

    @property
    def resident_bytes(self) -> int:
        return sum(self.scene_bytes.values())

    def _sample_memory(self):
        free, total = self.torch.cuda.mem_get_info()
        self.high_water = max(self.high_water, total - free)
        self.used_high_water = max(self.used_high_water, self._used())

    def _used(self) -> int:
        return self.resident_bytes + self.plan_bytes

    def _estimate(self, key) -> int:
        """Bytes of a new plan for the pair: the last plan made for it, else the library's estimate at a
        tile-key capacity of twice the (view, Gaussian) pairs per depth chunk (a generous first guess)."""
        if key in self.est:
            return self.est[key]
        scene, disp = self.scenes[key[0]], self.displays[key[1]]
        cap = max(self.min_keys.get(key, 0), 2 * disp.n_views * scene.n)
        H, W = disp.shape
        outs = (1 + (self.batch_max if self.batch_max > 1 else 0)) * H * W * 12
        return api.plan_estimate_bytes(scene, disp, self.opts, min(cap, 2**31 - 1)) + outs

    # ---- plans ----
    def _evict_for(self, need: int) -> bool:
        """Free idle plans (least recently used first) until `need` more bytes fit in the budget; evict nothing
        if even freeing every idle plan would not make room."""
        idle = sum(e.bytes for e in self.plans.values() if not e.busy)
        if self._used() - idle + need > self.budget:
            return False
        while self._used() + need > self.budget:
            victim = next((e for e in self.plans.values() if not e.busy), None)
            if victim is None:
                return False
            del self.plans[id(victim)]
            self.plan_bytes -= victim.bytes
            victim.plan.close()
            self.evicted += 1
        return True

    def _get_plan(self, key, stream, allow_more: bool = True):
        """An idle plan of the pair, or a new one; (None, reason) when the request has to wait.  A pair's first
        plan may evict idle plans of other pairs; further plans of a pair (for overlapping requests) are made only
        from unused budget, so busy pairs never push other pairs out."""
        have = False
        for e in self.plans.values():
            if e.key == key:
                have = True
                if not e.busy:
                    self.plans.move_to_end(id(e))
                    return e, None
        need = self._estimate(key)
        if have:
            if not allow_more or self._used() + need > self.budget:
                return None, "busy"
        elif not self._evict_for(need):
            return None, "memory"
        return self._new_plan(key, stream), None

    def warm(self, keys=None, log=None, probe_poses=(), copies: int = 1) -> None:
        """Create plans for the (scene, display) pairs (or those in `keys`) before timing, as far as the budget
        allows: one per pair first, then up to `copies` per pair from unused budget (so that requests of one pair can
        run side by side without a plan being made in the request loop).  Each plan is also run at `probe_poses`; a
        plan that overflows there is rebuilt with room for them."""
        keys = keys or [(s_, d) for s_ in self.scenes for d in self.displays]
        s = self.slots[0].stream
        made = []
        for copy in range(max(1, copies)):
            for k in keys:
                if copy > 0 and self._used() + self._estimate(k) > self.budget:
                    continue
                e = self._new_plan(k, s) if copy > 0 else self._get_plan(k, s)[0]
                if e is None:
                    break
                for attempt in range(3):
                    worst_ok, later = True, False
                    for c2w in probe_poses:
                        e.plan.launch(c2w, stream=s)
                        s.synchronize()
                        ok, need = e.plan.check()
                        self.min_keys[k] = max(self.min_keys.get(k, 0), need + need * 3 // 10 + 4096)
                        worst_ok &= ok
                        later |= e.plan.needs_all_chunks
                    if worst_ok:
                        break
                    if later:
                        # a probe pose needs a later depth chunk: the pair's plans keep every chunk
                        self.all_chunks.add(k)
                        e.plan.use_all_chunks(stream=s)
                        continue
                    del self.plans[id(e)]
                    self.plan_bytes -= e.bytes
                    e.plan.close()
                    e = self._new_plan(k, s)
                made.append(e)
                if log:
                    log("plan %s/%s (copy %d): %.2f GB" % (k[0], k[1], copy + 1, e.bytes / 2**30))
        self.torch.cuda.synchronize()

    def _new_plan(self, key, stream):
        """A new plan for the pair, unconditionally (the caller checked the budget)."""
        plan = api.Plan(self.ctx, self.scenes[key[0]], self.displays[key[1]], self.probe_c2w, opts=self.opts,
                        min_key_capacity=self.min_keys.get(key, 0), stream=stream)
        if self.batch_max > 1:
            plan.prepare_batch(self.batch_max, stream=stream)
        if key in self.all_chunks:
            plan.use_all_chunks(stream=stream)
        e = _PlanEntry(key, plan)
        self.est[key] = e.bytes
        self.plans[id(e)] = e
        self.plan_bytes += e.bytes
        self.created += 1
        self._sample_memory()
        return e

    def cancel(self, rid: int) -> None:
        """Drop request `rid` if it has not been launched yet (thread-safe; a launched frame runs to completion)."""
        with self._cancel_lock:
            self._cancel.add(rid)

    # ---- the loop ----
    def run(self, requests: list, realtime: bool = True, on_done=None) -> Report:
        """Serve `requests` (sorted by arrival).  With realtime=False every request is taken as already arrived.
        on_done(done) is called on the loop thread as each frame completes."""
        torch = self.torch
        pending = deque(dataclasses.replace(r) for r in sorted(requests, key=lambda r: r.arrival))
        queue: deque = deque()
        done: list = []
        cancelled: list = []
        stalled: list = []
        deferred_ids: set = set()  # waited for device memory
        waited_ids: set = set()  # waited for a busy plan of their pair
        replans = {}
        admitted = 0
        created0, evicted0 = self.created, self.evicted
        dog = Watchdog(self.watchdog_s) if self.watchdog_s else None
        # GPU completion times on the host clock: a reference event completes right before the host reads t_ref
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(self.slots[0].stream)
        ref.synchronize()
        t0 = time.perf_counter()
        t_ref = 0.0
        base = pending[0].arrival if pending else 0.0
        now = lambda: time.perf_counter() - t0  # noqa: E731
        while pending or queue or any(sl.reqs for sl in self.slots):
            t = now()
            while pending and (not realtime or pending[0].arrival - base <= t):
                r = pending.popleft()
                if not realtime:
                    r.arrival = base
                r.arrival -= base
                queue.append(r)
            if self._cancel:
                with self._cancel_lock:
                    drop = self._cancel & {r.rid for r in queue}
                    self._cancel -= drop
                if drop:
                    cancelled += sorted(drop)
                    queue = deque(r for r in queue if r.rid not in drop)
            # completions
            for sl in self.slots:
                if not sl.reqs or not sl.event.query():
                    continue
                t_done = t_ref + 1e-3 * ref.elapsed_time(sl.event)
                rs, e = sl.reqs, sl.entry
                if dog:
                    for r in rs:
                        dog.disarm(r.rid)
                ok, need = e.plan.check()
                e.busy = False
                sl.reqs, sl.entry = [], None
                # plans made later for this pair get 30% headroom over the largest chunk seen so far
                self.min_keys[e.key] = max(self.min_keys.get(e.key, 0), need + need * 3 // 10 + 4096)
                if not ok and e.plan.needs_all_chunks:
                    # a frame of a first-chunk plan needed a later depth chunk: the plan keeps every chunk from
                    # now on, and the requests are served again
                    self.all_chunks.add(e.key)
                    e.plan.use_all_chunks(stream=sl.stream)
                    for r in reversed(rs):
                        replans[r.rid] = replans.get(r.rid, 0) + 1
                        queue.appendleft(r)
                    sl.images = []
                    continue
                if not ok:
                    # a frame overflowed the plan's tile-key capacity: replace the plan and serve the requests again
                    del self.plans[id(e)]
                    self.plan_bytes -= e.bytes
                    e.plan.close()
                    for r in reversed(rs):
                        replans[r.rid] = replans.get(r.rid, 0) + 1
                        queue.appendleft(r)
                    sl.images = []
                    continue
                images = sl.images or [None] * len(rs)
                for r, img in zip(rs, images):
                    d = Done(r.rid, r.scene, r.display, r.arrival, sl.launched, max(t_done, sl.launched),
                             r.rid in deferred_ids, replans.get(r.rid, 0), img, len(rs))
                    done.append(d)
                    if on_done:
                        on_done(d)
                sl.images = []
            if dog:
                for rid, late in dog.poll(now()):
                    stalled.append((rid, late))
            # admissions, in arrival order, into free slots
            free = [sl for sl in self.slots if not sl.reqs]
            i = 0
            while free and i < len(queue):
                r = queue[i]
                sl = free[0]
                key = (r.scene, r.display)
                e, why = self._get_plan(key, sl.stream, allow_more=self.grow_in_loop)
                if e is None:
                    (deferred_ids if why == "memory" else waited_ids).add(r.rid)
                    i += 1
                    continue
                del queue[i]
                batch = [r]
                limit = min(self.batch_max, e.plan.batch_max)
                if limit > 1:
                    # later queued requests of the same pair join the launch, in arrival order
                    j = i
                    while j < len(queue) and len(batch) < limit:
                        if (queue[j].scene, queue[j].display) == key:
                            batch.append(queue[j])
                            del queue[j]
                        else:
                            j += 1
                free.pop(0)
                e.busy = True
                sl.reqs, sl.entry = batch, e
                sl.launched = now()
                if len(batch) == 1:
                    outs = [e.plan.launch(r.c2w, stream=sl.stream)]
                else:
                    outs = list(e.plan.launch_batch([b.c2w for b in batch], stream=sl.stream))
                if self.keep_images:
                    with torch.cuda.stream(sl.stream):
                        sl.images = [o.clone() for o in outs]
                sl.event.record(sl.stream)
                if dog:
                    for b in batch:
                        dog.arm(b.rid, sl.launched)
                admitted += len(batch)
            if queue and all(not sl.reqs for sl in self.slots):
                raise RuntimeError(f"request {queue[0].rid} ({queue[0].scene}, {queue[0].display}) does not fit in "
                                   f"the device-memory budget of {self.budget / 2**30:.2f} GiB")
            if not free or not queue:
                time.sleep(0)  # let the host breathe while frames run
        wall = max([d.finished for d in done] + [now() if not done else 0.0])
        with self._cancel_lock:
            self._cancel -= {r.rid for r in requests}   # cancellations of this run's requests are settled
        self._sample_memory()
        return Report(done=sorted(done, key=lambda d: d.rid), wall_s=wall, admitted=admitted,
                      deferred=len(deferred_ids), waited=len(waited_ids), replans=sum(replans.values()),
                      plans_created=self.created - created0,
                      plans_evicted=self.evicted - evicted0, hbm_high_water=self.high_water,
                      budget_high_water=self.used_high_water, budget=self.budget,
                      resident_bytes=self.resident_bytes, cancelled=cancelled, stalled=stalled)

    def close(self):
        torch = self.torch
        torch.cuda.synchronize()
        for e in list(self.plans.values()):
            e.plan.close()
        self.plans.clear()
        self.plan_bytes = 0
        for d in self.displays.values():
            d.close()
        for s in self.scenes.values():
            s.close()
