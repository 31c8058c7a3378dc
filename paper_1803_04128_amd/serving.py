"""Continuous-batching server for butterfly applies.

Many clients ask for g = K f with different operators (grid, phase, q,
amplitude, precision).  Building an operator's factors is the expensive
precomputation and is reused across inputs (Section 1 footnote and the
closing paragraph of Section 4 of arXiv:1803.04128); applying it is cheap per
vector and far more efficient in large batches.  The server therefore

* keeps built plans resident in device memory, in an LRU cache under an HBM
  budget that counts each plan's factors, workspace and staging buffers
  (admission: a plan that cannot fit, even after evicting every idle plan,
  is refused and its requests fail with AdmissionError);
* merges queued requests for the same plan into one apply of up to
  ``max_batch`` vectors (continuous batching: requests that arrive while a
  batch runs join the next batch of their plan; the plan of the oldest
  queued request goes next, so no plan starves);
* runs up to ``max_inflight`` batches at once, each on its own HIP stream,
  so batches of different plans overlap on the device, and timestamps every
  batch with a device event: a request's latency runs from its arrival to
  the completion of its batch on the GPU.

Scheduling and admission are host logic (``Scheduler``, ``PlanCache``) and
work with any plan object that has ``footprint`` and ``close()``; the device
side is ``ResidentPlan`` over the C ABI binding.  Staging copies into and out
of a plan's batch buffers are plain device copies; the transform itself runs
in the library's kernels.
"""

import collections
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Dict, List, Optional, Tuple

import numpy as np


class AdmissionError(RuntimeError):
    """The plan does not fit the HBM budget."""


class PinnedError(AdmissionError):
    """The plan fits the budget only once plans in use are released."""


@dataclass(frozen=True)
class PlanSpec:
    """An operator the server can build: the arguments of ``Plan``."""
    dim: int
    n: int
    phase: str
    params: Tuple[float, ...] = ()
    q: int = 8
    precision: str = "fp32"
    amplitude: Any = None        # None (alpha = 1) or (a, b), [r][N] arrays
    op: str = "N"                # "N", "T", "C" or "H": K, K^T, conj K, K^H

    @property
    def N(self):
        return self.n ** self.dim

    @property
    def r(self):
        return 1 if self.amplitude is None else len(self.amplitude[0])


@dataclass(eq=False)
class Request:
    rid: int
    plan: str                    # name the spec was registered under
    f: Any                       # device complex64 [nvec][N]
    arrival: float               # seconds after the start of the run
    out: Any = None              # device complex64 [nvec][N] (allocated
                                 # by the server when None)
    done: Optional[float] = None
    batch: int = -1
    error: Optional[str] = None

    @property
    def nvec(self):
        return 1 if self.f.dim() == 1 else int(self.f.shape[0])

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


class Scheduler:
    """Queue of requests in arrival order; forms batches of one plan."""

    def __init__(self, max_batch):
        if max_batch < 1:
            raise ValueError("max_batch must be >= 1")
        self.max_batch = max_batch
        self._q = collections.deque()

    def __len__(self):
        return len(self._q)

    def add(self, req):
        if req.nvec > self.max_batch:
            raise ValueError(f"request {req.rid}: {req.nvec} vectors > "
                             f"max_batch {self.max_batch}")
        self._q.append(req)

    def next_batch(self, busy=()):
        """(plan name, requests) for the plan of the oldest request whose
        plan is not in ``busy``: its queued requests in arrival order while
        the vectors fit max_batch (the first that does not fit ends the
        batch, which keeps each plan's requests in order).  None when no
        such request is queued."""
        name = next((r.plan for r in self._q if r.plan not in busy), None)
        if name is None:
            return None
        take, keep, total, full = [], collections.deque(), 0, False
        for r in self._q:
            if r.plan == name and not full:
                if total + r.nvec <= self.max_batch:
                    take.append(r)
                    total += r.nvec
                    continue
                full = True
            keep.append(r)
        self._q = keep
        return name, take

    def drop(self, name):
        """Remove and return every queued request of a plan."""
        out = [r for r in self._q if r.plan == name]
        self._q = collections.deque(r for r in self._q if r.plan != name)
        return out


class PlanCache:
    """Resident plans under an HBM budget, least recently used evicted first.

    footprint(name) gives the device bytes a plan will hold, computed on the
    host before anything is allocated; build(name) returns an object with
    ``footprint`` (the bytes it holds) and ``close()``.  Admission checks
    the budget and evicts before building, so device memory never holds
    more than the budget and each admission builds once.  A plan in
    ``pinned`` (in use by the caller) is never evicted.  A build that fails
    (a library error such as an allocation failure) is an admission failure
    of that plan only."""

    def __init__(self, budget_bytes, build: Callable[[str], Any],
                 footprint: Callable[[str], int]):
        self.budget = int(budget_bytes)
        self._build = build
        self._footprint = footprint
        self._res = collections.OrderedDict()
        self.builds = 0
        self.evictions = 0

    @property
    def resident_bytes(self):
        return sum(p.footprint for p in self._res.values())

    def names(self):
        return list(self._res)

    def get(self, name, pinned=()):
        if name in self._res:
            self._res.move_to_end(name)
            return self._res[name]
        try:
            need = int(self._footprint(name))
        except Exception as e:        # a spec the library refuses
            raise AdmissionError(f"plan {name}: {e}") from e
        if need > self.budget:
            raise AdmissionError(f"plan {name}: {need} bytes > budget "
                                 f"{self.budget}")
        idle = [v for v in self._res if v not in pinned]
        if self.resident_bytes - sum(self._res[v].footprint for v in idle) \
                + need > self.budget:
            raise PinnedError(f"plan {name}: no room next to pinned plans")
        for victim in idle:
            if self.resident_bytes + need <= self.budget:
                break
            self._res.pop(victim).close()
            self.evictions += 1
        try:
            obj = self._build(name)
        except Exception as e:
            raise AdmissionError(f"plan {name}: build failed: {e}") from e
        self.builds += 1
        if self.resident_bytes + obj.footprint > self.budget:
            # the estimate was short: never keep more than the budget
            obj.close()
            raise AdmissionError(f"plan {name}: holds {obj.footprint} bytes, "
                                 f"estimated {need}")
        self._res[name] = obj
        return obj

    def clear(self):
        while self._res:
            self._res.popitem(last=False)[1].close()


class ResidentPlan:
    """A device-resident plan with staging buffers for batches of up to
    max_batch vectors."""

    def __init__(self, spec: PlanSpec, max_batch):
        import torch
        from . import Plan
        self.spec = spec
        self.plan = Plan(spec.dim, spec.n, spec.phase, spec.params, q=spec.q,
                         amplitude=spec.amplitude, precision=spec.precision,
                         max_nvec=max_batch, op=spec.op)
        self.fin = torch.empty((max_batch, spec.N), dtype=torch.complex64,
                               device="cuda")
        self.fout = torch.empty_like(self.fin)
        info = self.plan.info()
        # factor_bytes covers every device allocation of the plan (factors,
        # amplitude, stored switch blocks, low-rank phase factors)
        self.footprint = (info["factor_bytes"] + info["workspace_bytes"] +
                          2 * self.fin.numel() * 8)

    @staticmethod
    def footprint_of(spec: PlanSpec, max_batch):
        """Device bytes of ResidentPlan(spec, max_batch), from the host
        (bf_plan_footprint plus the two staging buffers)."""
        from . import plan_footprint
        return (plan_footprint(spec.dim, spec.n, spec.phase, spec.params,
                               q=spec.q, amplitude=spec.amplitude,
                               precision=spec.precision, max_nvec=max_batch,
                               op=spec.op) +
                2 * max_batch * spec.N * 8)

    def run(self, reqs, stream):
        """Stage the requests' vectors, apply once, copy results out, all on
        ``stream``."""
        import torch
        with torch.cuda.stream(stream):
            off = 0
            for r in reqs:
                self.fin[off:off + r.nvec].copy_(r.f.reshape(r.nvec, -1))
                off += r.nvec
            self.plan.apply(self.fin[:off], out=self.fout[:off],
                            stream=stream)
            off = 0
            for r in reqs:
                r.out.reshape(r.nvec, -1).copy_(self.fout[off:off + r.nvec])
                off += r.nvec

    def close(self):
        self.plan.close()
        self.fin = self.fout = None


class Server:
    """Open-loop serving run over a list of requests with arrival times."""

    def __init__(self, hbm_budget_bytes=64 << 30, max_batch=64,
                 max_inflight=2, poll_s=50e-6):
        self.specs: Dict[str, PlanSpec] = {}
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.poll_s = poll_s
        self.cache = PlanCache(hbm_budget_bytes, self._build,
                               self._footprint)
        self.batches: List[Tuple[str, int]] = []
        # device intervals of the batches: (start s, end s, plan, slot)
        self.intervals: List[Tuple[float, float, str, int]] = []

    def register(self, name, spec: PlanSpec):
        self.specs[name] = spec

    def _build(self, name):
        return ResidentPlan(self.specs[name], self.max_batch)

    def _footprint(self, name):
        return ResidentPlan.footprint_of(self.specs[name], self.max_batch)

    def run(self, requests: List[Request]):
        """Serve every request; fills done (seconds from the run's start),
        batch and error.  Returns the requests in arrival order.

        Each of the max_inflight slots owns a HIP stream (default priority);
        batches of different plans run concurrently on the device, and a
        plan is in flight on at most one slot at a time (its staging buffers
        and workspace are its own)."""
        import torch
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            if r.plan not in self.specs:
                raise KeyError(f"request {r.rid}: unknown plan {r.plan}")
            if r.out is None:
                r.out = torch.empty_like(r.f)
        sched = Scheduler(self.max_batch)
        main = torch.cuda.current_stream()
        slots = [torch.cuda.Stream() for _ in range(self.max_inflight)]
        for st in slots:
            st.wait_stream(main)        # inputs written on the caller's stream
        torch.cuda.synchronize()
        base = torch.cuda.Event(enable_timing=True)
        base.record(main)
        t0 = time.perf_counter()
        inflight = {}       # slot -> (start event, end event, batch, plan)
        i, nb = 0, 0

        def retire(slot):
            ev0, ev, batch, name = inflight.pop(slot)
            t = base.elapsed_time(ev) / 1e3
            self.intervals.append((base.elapsed_time(ev0) / 1e3, t, name,
                                   slot))
            for r in batch:
                r.done = t

        def drain():
            for slot in list(inflight):
                inflight[slot][1].synchronize()
                retire(slot)

        while i < len(reqs) or len(sched) or inflight:
            now = time.perf_counter() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                sched.add(reqs[i])
                i += 1
            for slot in list(inflight):
                if inflight[slot][1].query():
                    retire(slot)
            free = [k for k in range(len(slots)) if k not in inflight]
            busy = {v[3] for v in inflight.values()}
            nxt = sched.next_batch(busy=busy) if (free and len(sched)) else None
            if nxt is not None:
                name, batch = nxt
                try:
                    try:
                        rp = self.cache.get(name, pinned=busy)
                    except PinnedError:
                        # room only once the plans in flight are released
                        drain()
                        free = list(range(len(slots)))
                        rp = self.cache.get(name)
                except AdmissionError as e:
                    for r in batch + sched.drop(name):
                        r.error = str(e)
                    continue
                slot = free[0]
                ev0 = torch.cuda.Event(enable_timing=True)
                ev0.record(slots[slot])
                rp.run(batch, slots[slot])
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(slots[slot])
                for r in batch:
                    r.batch = nb
                nb += 1
                self.batches.append((name, sum(r.nvec for r in batch)))
                inflight[slot] = (ev0, ev, batch, name)
                continue
            # nothing to launch now: wait for an arrival or a completion
            wait = (reqs[i].arrival - (time.perf_counter() - t0)
                    if i < len(reqs) else float("inf"))
            if inflight:
                wait = min(wait, self.poll_s)
            if wait > 0 and wait != float("inf"):
                time.sleep(wait)
        torch.cuda.synchronize()
        return reqs

    def close(self):
        self.cache.clear()


def summarize(reqs, N_of):
    """Latency percentiles (ms) and throughput (N * nvec / s) of a run.
    N_of(plan name) gives the plan's N."""
    ok = [r for r in reqs if r.error is None and r.done is not None]
    lat = np.array([r.latency for r in ok]) * 1e3
    if not ok:
        return dict(served=0, failed=len(reqs))
    span = max(r.done for r in ok) - min(r.arrival for r in ok)
    work = sum(N_of(r.plan) * r.nvec for r in ok)
    return dict(served=len(ok), failed=len(reqs) - len(ok),
                p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)),
                mean_ms=float(lat.mean()),
                throughput=work / span if span > 0 else float("nan"),
                span_s=span)


def overlap_fraction(intervals):
    """Fraction of the busy device time during which at least two batches
    were running (from the batches' start and end events)."""
    ev = sorted([(a, 1) for a, _, _, _ in intervals] +
                [(b, -1) for _, b, _, _ in intervals])
    busy = multi = 0.0
    depth, last = 0, None
    for t, d in ev:
        if last is not None and depth > 0:
            busy += t - last
            if depth > 1:
                multi += t - last
        depth += d
        last = t
    return multi / busy if busy > 0 else 0.0
