"""Continuous-batching reconstruction server.

Requests (a target descriptor, a start field and a spec) arrive over time.
Requests with the same spec (shape, channels, levels, displacements) share a
*group*: one batched solver of B slots whose field, target and L-BFGS history
stay resident in HBM.  Each scheduler tick

  1. admits waiting requests into free slots of their group, creating a group
     only when its HBM footprint fits the budget (otherwise the request waits,
     and idle groups are released to make room);
  2. advances every group with running slots by a few L-BFGS iterations, each
     group on its own stream in its own host thread so that the groups' kernels
     overlap on the device;
  3. retires slots that reached the error tolerance or the iteration cap and
     records latency from arrival to result.

With asynchronous=True the groups do not wait for each other: a group is
advanced again as soon as its own iterations finish, and requests are admitted
into a group only between its advances.  A group of small fields then keeps
iterating while a group of 256^3 fields works through its slower iterations,
instead of idling to the end of a common tick.

A request may carry a timeout (seconds from arrival) and may be cancelled
(Server.cancel); either retires it at the next scheduling point of its group,
with status TIMED_OUT or CANCELLED, the slot freed for the next request.

A slot's iterates do not depend on the other slots (see dmcr_solver_iterate),
so a request's result is the same alone and in the mix.  The scheduler is
written against a small executor interface so that its policy can be tested
on the CPU with a simulated executor.
"""
import concurrent.futures as cf
import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

# server-side outcomes (library statuses are >= -5): admission impossible, the
# request's timeout passed, or the caller cancelled it
NO_FIT, TIMED_OUT, CANCELLED = -2, -100, -101


@dataclass
class Request:
    rid: int
    arrival: float                     # seconds after the stream starts
    key: Tuple                         # group key: (shape, channels, levels, max_disp)
    voxels: int                        # finest-level voxels (all channels)
    payload: object = None             # executor-specific (target descriptor, start field)
    timeout: Optional[float] = None    # seconds after arrival; None: no limit
    target_E0: Optional[float] = None  # E of a zero descriptor against the target (its weighted norm)
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    final_E: Optional[float] = None
    iters: int = 0
    status: Optional[int] = None

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.arrival


class Group:
    """Executor-side batch of slots for one key (interface)."""
    key: Tuple
    capacity: int
    footprint: int

    def admit(self, slot: int, req: Request) -> None: ...
    def step(self, iterations: int) -> List[Tuple[int, int, float, int]]: ...   # (slot, status, E, iters) finished
    def cancel(self, slot: int) -> Tuple[float, int]: ...   # stop a slot between steps: (E, iters) so far
    def release(self) -> None: ...


class Executor:
    def footprint(self, key, capacity) -> int: ...
    def capacity(self, key) -> int: ...
    def make_group(self, key, capacity) -> Group: ...
    def now(self) -> float: ...


class Server:
    def __init__(self, executor: Executor, budget_bytes: int, iters_per_tick: int = 4, threads: int = 8,
                 asynchronous: bool = False):
        self.asynchronous = asynchronous
        self.ex = executor
        self.budget = budget_bytes
        self.iters_per_tick = iters_per_tick
        self.groups: Dict[Tuple, Group] = {}
        self.free: Dict[Tuple, List[int]] = {}
        self.owner: Dict[Tuple, Dict[int, Request]] = {}
        self.queue: List[Request] = []
        self.done: List[Request] = []
        self.pool = cf.ThreadPoolExecutor(max_workers=threads)
        self.peak_bytes = 0
        self.ticks = 0
        self.cancelled = set()

    # -- memory ----------------------------------------------------------------
    def used(self) -> int:
        return sum(g.footprint for g in self.groups.values())

    def _release_idle(self, need: int, keep_key) -> bool:
        for k in list(self.groups):
            if k == keep_key or self.owner[k]:
                continue
            if any(r.key == k for r in self.queue):
                continue
            self.groups[k].release()
            del self.groups[k], self.free[k], self.owner[k]
            if self.used() + need <= self.budget:
                return True
        return self.used() + need <= self.budget

    def _group_for(self, key) -> Optional[Group]:
        if key in self.groups:
            return self.groups[key]
        cap = self.ex.capacity(key)
        while cap >= 1:
            need = self.ex.footprint(key, cap)
            if self.used() + need <= self.budget or self._release_idle(need, key):
                g = self.ex.make_group(key, cap)
                self.groups[key] = g
                self.free[key] = list(range(cap))
                self.owner[key] = {}
                self.peak_bytes = max(self.peak_bytes, self.used())
                return g
            cap //= 2
        return None

    # -- scheduling ------------------------------------------------------------
    def submit(self, req: Request):
        self.queue.append(req)

    def cancel(self, rid: int):
        """Cancel a queued or running request: it is retired with CANCELLED at the next
        scheduling point of its group (never while the group is being advanced)."""
        self.cancelled.add(rid)

    def _dead(self, req: Request, now: float):
        if req.rid in self.cancelled:
            return CANCELLED
        if req.timeout is not None and now - req.arrival > req.timeout:
            return TIMED_OUT
        return None

    def _expire(self, busy=()):
        """Retire cancelled and timed-out requests: queued ones at once, running ones
        of groups that are not being advanced (their slot is stopped and freed)."""
        now = self.ex.now()
        waiting = []
        for req in self.queue:
            why = self._dead(req, now)
            if why is None:
                waiting.append(req)
                continue
            req.t_done, req.status, req.final_E = now, why, float("nan")
            self.done.append(req)
        self.queue = waiting
        for k, owners in self.owner.items():
            if k in busy:
                continue
            for slot, req in list(owners.items()):
                why = self._dead(req, now)
                if why is None:
                    continue
                req.final_E, req.iters = self.groups[k].cancel(slot)
                req.t_done, req.status = now, why
                del owners[slot]
                self.free[k].append(slot)
                self.done.append(req)

    def next_deadline(self):
        """Earliest timeout among queued and running requests (executor clock), or None."""
        ts = [r.arrival + r.timeout for r in self.queue if r.timeout is not None]
        ts += [r.arrival + r.timeout for o in self.owner.values() for r in o.values() if r.timeout is not None]
        return min(ts) if ts else None

    def _admit(self, busy=()):
        """Admit queued requests into free slots; groups in `busy` are being advanced
        and take no requests until they return."""
        waiting = []
        for req in self.queue:
            if req.key in busy:
                waiting.append(req)
                continue
            g = self._group_for(req.key)
            if g is None and not self.groups and self.ex.footprint(req.key, 1) > self.budget:
                # can never fit, even alone: fail it instead of waiting forever
                req.t_done, req.status, req.final_E = self.ex.now(), NO_FIT, float("nan")
                self.done.append(req)
                continue
            if g is None or not self.free[req.key]:
                waiting.append(req)
                continue
            slot = self.free[req.key].pop(0)
            req.t_admit = self.ex.now()
            g.admit(slot, req)
            self.owner[req.key][slot] = req
        self.queue = waiting

    def _retire(self, k, finished):
        for slot, status, E, iters in finished:
            req = self.owner[k].pop(slot)
            req.t_done = self.ex.now()
            req.final_E, req.iters, req.status = E, iters, status
            self.done.append(req)
            self.free[k].append(slot)

    def tick(self):
        self._expire()
        self._admit()
        busy = [k for k in self.groups if self.owner[k]]
        futs = {self.pool.submit(self.groups[k].step, self.iters_per_tick): k for k in busy}
        for f in cf.as_completed(futs):
            self._retire(futs[f], f.result())
        self.ticks += 1
        hook = getattr(self.ex, "after_tick", None)
        if hook:
            hook()

    def idle(self):
        return not self.queue and not any(self.owner[k] for k in self.groups)

    def run(self, requests: List[Request], wait=None):
        """Release requests at their arrival times (executor clock) and serve until all finish."""
        if self.asynchronous:
            return self._run_async(requests, wait)
        pending = sorted(requests, key=lambda r: r.arrival)
        i = 0
        t0 = self.ex.now()
        while i < len(pending) or not self.idle():
            now = self.ex.now() - t0
            while i < len(pending) and pending[i].arrival <= now:
                r = pending[i]
                r.arrival += t0
                self.submit(r)
                i += 1
            if self.idle() and i < len(pending):
                (wait or self.ex.wait_until)(t0 + pending[i].arrival)
                continue
            self.tick()
        return self.done

    def _run_async(self, requests: List[Request], wait=None):
        pending = sorted(requests, key=lambda r: r.arrival)
        i = 0
        t0 = self.ex.now()
        running: Dict[Tuple, cf.Future] = {}
        while i < len(pending) or self.queue or running or any(self.owner[k] for k in self.groups):
            now = self.ex.now() - t0
            while i < len(pending) and pending[i].arrival <= now:
                r = pending[i]
                r.arrival += t0
                self.submit(r)
                i += 1
            self._expire(busy=running)
            self._admit(busy=running)
            for k in self.groups:
                if self.owner[k] and k not in running:
                    running[k] = self.pool.submit(self.groups[k].step, self.iters_per_tick)
            if not running:
                if i < len(pending):
                    (wait or self.ex.wait_until)(t0 + pending[i].arrival)
                    continue
                if self.queue:
                    raise RuntimeError("%d requests can be neither admitted nor failed" % len(self.queue))
                break
            wake = [t0 + pending[i].arrival] if i < len(pending) else []
            dl = self.next_deadline()
            if dl is not None:
                wake.append(dl)
            timeout = max(0.0, min(wake) - self.ex.now()) if wake else None
            finished, _ = cf.wait(list(running.values()), timeout=timeout, return_when=cf.FIRST_COMPLETED)
            for k in [k for k, f in running.items() if f in finished]:
                self._retire(k, running.pop(k).result())
                self.ticks += 1
        return self.done

    def close(self):
        for g in self.groups.values():
            g.release()
        self.groups.clear()
        self.pool.shutdown()


def summary(done: List[Request]):
    """Throughput, latency percentiles (arrival to result) and per-request figures of
    the requests that ran to an end (converged or out of iterations); requests that
    were cancelled, timed out or could not fit are counted apart.  rel_err is the
    paper-style relative error |D - D_des| / |D_des| of the weighted multigrid
    descriptor, sqrt(E / E0) with E0 the error of a zero descriptor."""
    ran = [r for r in done if r.status is not None and r.status >= -5 and r.status != NO_FIT]
    lat = np.array([r.latency for r in ran]) if ran else np.zeros(1)
    t0 = min(r.arrival for r in done)
    t1 = max(r.t_done for r in done)
    vox_it = sum(r.voxels * r.iters for r in done)
    iters = np.array([r.iters for r in ran]) if ran else np.zeros(1)
    out = dict(requests=len(done), makespan_s=t1 - t0, requests_per_s=len(ran) / (t1 - t0),
               voxel_it_per_s=vox_it / (t1 - t0), p50_s=float(np.percentile(lat, 50)),
               p99_s=float(np.percentile(lat, 99)), mean_s=float(lat.mean()),
               converged=int(sum(1 for r in done if r.status == 0)),
               max_final_E=float(max(r.final_E for r in ran)) if ran else float("nan"),
               iters_mean=float(iters.mean()), iters_p50=float(np.percentile(iters, 50)),
               iters_p99=float(np.percentile(iters, 99)),
               cancelled=sum(1 for r in done if r.status == CANCELLED),
               timed_out=sum(1 for r in done if r.status == TIMED_OUT),
               no_fit=sum(1 for r in done if r.status == NO_FIT))
    rel = [math.sqrt(r.final_E / r.target_E0) for r in ran if r.target_E0]
    if rel:
        out.update(rel_err_p50=float(np.percentile(rel, 50)), rel_err_max=float(max(rel)))
    return out


# ---------------------------------------------------------------------------
# GPU executor (libdmcr solver slots)
# ---------------------------------------------------------------------------
class GpuGroup(Group):
    def __init__(self, key, capacity, bounds, opt):
        import torch
        from . import dmcr
        self.torch, self.dmcr = torch, dmcr
        shape, C, L, P = key
        self.key, self.capacity = key, capacity
        self.spec = dmcr.Spec(shape=shape, n_channels=C, n_levels=L, max_disp=P)
        self.stream = torch.cuda.Stream()
        # the solver's buffers are allocated (and cleared) in the order of self.stream
        self.solver = dmcr.Solver(self.spec, capacity, bounds, opt, stream=self.stream)
        self.footprint = self.solver.footprint
        self.started: List[int] = []
        self.keep = False
        self.fields = {}          # kept result fields by slot (the latest request of each slot)
        self.fields_by_rid = {}   # and by request id
        self.rid_of = {}

    def admit(self, slot, req):
        S_target, start = req.payload
        self.rid_of[slot] = req.rid
        # the target was produced on the admitting thread's stream
        self.stream.wait_stream(self.torch.cuda.current_stream())
        with self.torch.cuda.stream(self.stream):
            start.fill(self.solver.phi[slot])
            self.solver.St[slot].copy_(S_target, non_blocking=True)
        S_target.record_stream(self.stream)
        self.solver.slots[slot].active = 0
        self.started.append(slot)

    def cancel(self, slot):
        if slot in self.started:          # admitted, not yet started
            self.started.remove(slot)
            return float("nan"), 0
        s = self.solver.slots[slot]
        s.active = 0
        return s.E, s.iters

    def step(self, iterations):
        torch = self.torch
        with torch.cuda.stream(self.stream):
            if self.started:
                self.solver.start(self.started, stream=self.stream)
                self.started = []
            self.solver.iterate(iterations, stream=self.stream)
        out = []
        for b in range(self.capacity):
            s = self.solver.slots[b]
            if s.active and s.status != self.dmcr.RUNNING:
                if self.keep:
                    with torch.cuda.stream(self.stream):
                        self.fields[b] = self.solver.phi[b].detach().clone()
                    self.fields_by_rid[self.rid_of[b]] = self.fields[b]
                out.append((b, s.status, s.E, s.iters))
                s.active = 0
        return out

    def release(self):
        self.solver = None


class GpuExecutor(Executor):
    def __init__(self, bounds=None, opt=None, max_slots=None, keep_fields=False):
        import torch
        from . import dmcr
        self.dmcr, self.torch = dmcr, torch
        self.keep_fields = keep_fields
        self.bounds = bounds or dmcr.Bounds()
        self.opt = opt or dmcr.Opt(max_iter=2000, tol_derr=1e-4)
        self.max_slots = max_slots

    def capacity(self, key):
        shape, C, L, P = key
        vox = int(np.prod(shape)) * C
        cap = max(1, min(32, (1 << 22) // vox))   # about 4M voxels per group
        return min(cap, self.max_slots) if self.max_slots else cap

    def footprint(self, key, capacity):
        shape, C, L, P = key
        spec = self.dmcr.Spec(shape=shape, n_channels=C, n_levels=L, max_disp=P)
        K = self.dmcr.dmcr_descriptor_size(spec)
        return (self.dmcr.dmcr_reconstruct_workspace_size(spec, capacity, self.opt) + 256 +
                capacity * (int(np.prod(shape)) * C * 4 + K * 8))

    def make_group(self, key, capacity):
        g = GpuGroup(key, capacity, self.bounds, self.opt)
        g.keep = self.keep_fields
        return g

    def now(self):
        return time.perf_counter()

    def wait_until(self, t):
        d = t - time.perf_counter()
        if d > 0:
            time.sleep(min(d, 0.01))


# ---------------------------------------------------------------------------
# the serving workload: Poisson stream of mixed 2-D / 3-D, 2- and 3-phase requests
# ---------------------------------------------------------------------------
SIZES = [(128, 128), (256, 256), (512, 512), (1024, 1024), (64, 64, 64), (128, 128, 128), (256, 256, 256)]


def make_key(shape, phases):
    """P = 31 in 2-D, 16 in 3-D; n_levels 0 lets the library apply the paper's level
    rule (Appendix B: coarsest side about 2 (P + 1)) and clip P per level."""
    P = 31 if len(shape) == 2 else 16
    return (tuple(shape), phases - 1, 0, (P,))


def request_stream(n, rate, seed=0, sizes=SIZES):
    """(arrival, shape, phases, generator, seed) for a Poisson stream of n requests."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        shape = sizes[rng.integers(len(sizes))]
        phases = int(rng.integers(2, 4))
        gen = ("boolean", "grf")[rng.integers(2)]
        out.append((t, shape, phases, gen, int(rng.integers(1 << 30))))
    return out


def target_field(shape, phases, gen, seed):
    """Seeded target microstructure [phases-1][shape] from the synthetic generators."""
    from . import synth
    d = len(shape)
    if gen == "boolean":
        if phases == 2:
            return synth.boolean_spheres(shape, 4 if d == 2 else 6, 0.30, seed)[0]
        semi = (8, 3) if d == 2 else (10, 4, 4)
        return synth.spheres_and_ellipsoids(shape, 4 if d == 2 else 6, 0.20, semi, 0.15, seed)[0]
    ell = 12 if min(shape) >= 128 else 6
    if phases == 2:
        return synth.grf_two_phase(shape, ell, 0.40, seed)
    return synth.grf_three_phase(shape, ell, 0.25, 0.20, seed)


class TargetCache:
    """Target descriptors per (key, generator, variant), computed on the GPU from the
    seeded target microstructures (two variants per class), with E0, the error of a
    zero descriptor against each (the target's weighted norm, for relative errors)."""

    def __init__(self, variants=2):
        self.variants = variants
        self.cache = {}

    def get(self, key, shape, phases, gen, seed):
        import torch
        from . import dmcr
        v = seed % self.variants
        ck = (key, gen, v)
        if ck not in self.cache:
            f = target_field(shape, phases, gen, 1000 + 17 * v + 3 * phases).astype(np.float32)
            spec = dmcr.Spec(shape=key[0], n_channels=key[1], n_levels=key[2], max_disp=key[3])
            S = dmcr.dmcr_descriptor_forward(spec, torch.from_numpy(f[None]).cuda())
            E0, _ = dmcr.dmcr_error_cotangent(spec, torch.zeros_like(S), S.double())
            self.cache[ck] = (S[0].double(), float(E0.item()))
        return self.cache[ck]


class SeededStart:
    """Start field of a request: U(0,1) per channel, scaled by 1/C so the phase
    indicators start with a sum <= 1; drawn on the device from the request seed."""

    def __init__(self, seed, channels):
        self.seed, self.channels = seed, channels

    def fill(self, out):
        import torch
        g = torch.Generator(device=out.device)
        g.manual_seed(self.seed)
        out.uniform_(0.0, 1.0, generator=g)
        if self.channels > 1:
            out.mul_(1.0 / self.channels)
        return out


def gpu_requests(stream, cache: TargetCache):
    out = []
    for i, (t, shape, phases, gen, seed) in enumerate(stream):
        key = make_key(shape, phases)
        S, E0 = cache.get(key, shape, phases, gen, seed)
        out.append(Request(rid=i, arrival=t, key=key, voxels=int(np.prod(shape)) * (phases - 1),
                           payload=(S, SeededStart(seed, phases - 1)), target_E0=E0))
    return out


def sequential_buffers(requests, opt=None):
    """Per class: spec, field, target and workspace of a batch-1 reconstruction,
    allocated once up front so that the one-at-a-time baseline allocates nothing
    while it runs."""
    import torch
    from . import dmcr
    opt = opt or dmcr.Opt(max_iter=2000, tol_derr=1e-4)
    bufs = {}
    for r in requests:
        if r.key in bufs:
            continue
        shape, C, L, P = r.key
        spec = dmcr.Spec(shape=shape, n_channels=C, n_levels=L, max_disp=P)
        phi = torch.empty((1, C) + tuple(shape), dtype=torch.float32, device="cuda")
        St = torch.empty((1, dmcr.dmcr_descriptor_size(spec)), dtype=torch.float64, device="cuda")
        ws = dmcr.workspace(dmcr.dmcr_reconstruct_workspace_size(spec, 1, opt))
        bufs[r.key] = (spec, phi, St, ws)
    return bufs


def run_sequential(requests, bounds=None, opt=None, bufs=None, keep_fields=False):
    """Plain one-at-a-time GPU reconstruction (batch 1, no overlap), in arrival order,
    with all requests available at the start and every class's buffers resident.
    Returns the finished requests (and their fields with keep_fields)."""
    from . import dmcr
    bounds = bounds or dmcr.Bounds()
    opt = opt or dmcr.Opt(max_iter=2000, tol_derr=1e-4)
    bufs = bufs if bufs is not None else sequential_buffers(requests, opt)
    fields = {}
    t0 = time.perf_counter()
    for r in sorted(requests, key=lambda r: r.arrival):
        spec, phi, St, ws = bufs[r.key]
        S, start = r.payload
        start.fill(phi[0])
        St[0].copy_(S)
        code, res = dmcr.dmcr_reconstruct(spec, St, phi, bounds, opt, ws)
        r.arrival, r.t_admit, r.t_done = t0, t0, time.perf_counter()
        r.final_E, r.iters, r.status = res[0]["final_E"], res[0]["iters"], res[0]["why"]
        if keep_fields:
            fields[r.rid] = phi[0].clone()
    return (requests, fields) if keep_fields else requests


def rounded_errors(requests, fields):
    """E of each result field thresholded at 0.5 (the rounded field of Sec. 5.1,
    Fig. 5) against the request's target, and its relative error sqrt(E / E0)."""
    import torch
    from . import dmcr
    out = {}
    for r in requests:
        if r.rid not in fields:
            continue
        shape, C, L, P = r.key
        spec = dmcr.Spec(shape=shape, n_channels=C, n_levels=L, max_disp=P)
        binary = (fields[r.rid] > 0.5).to(torch.float32)[None].contiguous()
        S = dmcr.dmcr_descriptor_forward(spec, binary)
        E, _ = dmcr.dmcr_error_cotangent(spec, S, r.payload[0][None].contiguous())
        e = float(E.item())
        out[r.rid] = (e, math.sqrt(e / r.target_E0) if r.target_E0 else float("nan"))
    return out
