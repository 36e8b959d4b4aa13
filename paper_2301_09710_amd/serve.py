"""Continuous-batching EM reconstruction service on one GPU.

Requests are ML-EM reconstructions (Sec. II-B, Eq. (7)-(8) with beta -> 0) of
uneven sizes: each carries its own attenuation map, PSFs, sinogram and
background, and asks for a number of EM iterations.  The service keeps every
admitted request's images, sinograms and PSFs resident in HBM, admits
requests by memory (the plan workspace from ``spect_workspace_bytes`` plus
the request's own buffers) and by free slots, and advances all admitted
requests one EM iteration at a time on their own HIP streams, so their work
overlaps on the device.  A request that arrives while others run is admitted
as soon as a slot and enough memory free up -- between iterations, not after
the batch ends.

``Scheduler`` is the admission and accounting logic alone (no GPU), so that
it can be tested on the CPU; ``GpuExecutor`` runs the requests on libspect;
``serve`` drives both over an arrival trace and reports per-request latency
(arrival to result on the host), p50 / p99 and throughput.

All projector work runs in libspect's kernels; torch supplies device memory,
streams and events.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Deque, Dict, List, Optional

import numpy as np

from . import spect, synth

# ---------------------------------------------------------------- requests

SIZES = ("serve64", "serve96", "paper")


@dataclasses.dataclass
class Request:
    rid: int
    size: str                 # a synth.CONFIGS name
    seed: int
    arrival: float            # seconds after the start of the trace
    iters: int = 8
    precision: str = "fp32"
    method: str = "direct"    # PSF convolution: "direct" or "fft" (FP32 only)


@dataclasses.dataclass
class Done:
    rid: int
    size: str
    arrival: float
    admitted: float
    finished: float
    x: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def poisson_trace(n: int, rate: float, seed: int = 0, iters: int = 8,
                  sizes=SIZES, precision: str = "fp32", method: str = "direct") -> List[Request]:
    """n requests with exponential inter-arrival times (mean 1/rate) and sizes
    drawn uniformly from ``sizes``; each request's phantom, attenuation map
    and Poisson data come from its own seed."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    pick = rng.integers(0, len(sizes), size=n)
    return [Request(i, sizes[int(pick[i])], seed * 100003 + i, float(t[i]), iters, precision, method)
            for i in range(n)]


def geometry_of(size: str):
    c = synth.CONFIGS[size]
    return c["nx"], c["ny"], c["nz"], c["nview"], c["px"], c["pz"], c["dy"]


# The caching allocator rounds every device buffer above 1 MiB up to a
# multiple of 2 MiB; a request holds eight buffers.
ALLOC_ROUND = 2 << 20
REQUEST_BUFFERS = 8


def request_bytes(size: str, precision: str = "fp32", cache_mubar: bool = True,
                  method: str = "direct") -> int:
    """Device memory one admitted request holds: the plan workspace and the
    request's buffers (mu, PSFs, sinogram, background, image, sensitivity and
    the projection of ones the sensitivity is made from), each rounded up as
    the caching allocator rounds it."""
    nx, ny, nz, nview, px, pz, dy = geometry_of(size)
    g, _ = spect.make_geom(nx, ny, nz, nview, px, pz, dy,
                           flags=(spect.SPECT_CACHE_MUBAR if cache_mubar else 0) |
                           spect.METHODS[method],
                           conv_precision=spect.PRECISIONS[precision])
    N, M = nx * ny * nz, nview * nz * nx
    bufs = [spect.spect_workspace_bytes(g), 4 * N, 4 * N, 4 * N, 4 * M, 4 * M, 4 * M,
            4 * nview * ny * pz * px]
    assert len(bufs) == REQUEST_BUFFERS
    return sum(-(-b // ALLOC_ROUND) * ALLOC_ROUND for b in bufs)


# ---------------------------------------------------------------- scheduler

class Scheduler:
    """Admission by free slots and a memory budget, first come first served.

    ``need(req)`` gives the bytes a request holds while admitted.  A request
    whose need exceeds the whole budget can never run and is rejected when it
    reaches the head of the queue.  ``bypass`` lets up to that many later
    requests that fit go ahead of a head that does not fit yet (0: strict
    FIFO), which keeps small requests flowing while a large one waits."""

    def __init__(self, budget_bytes: int, max_slots: int, need: Callable[[Request], int],
                 bypass: int = 0):
        if budget_bytes <= 0 or max_slots <= 0:
            raise ValueError("budget and slots must be positive")
        self.budget, self.max_slots, self.need, self.bypass = budget_bytes, max_slots, need, bypass
        self.queue: Deque[Request] = collections.deque()
        self.active: Dict[int, int] = {}          # rid -> bytes held
        self.rejected: List[int] = []
        self.in_use = 0
        self.peak = 0

    def arrive(self, req: Request) -> None:
        self.queue.append(req)

    def admit(self) -> List[Request]:
        """Requests admitted now (removed from the queue, memory reserved)."""
        out = []
        skipped = 0
        i = 0
        while i < len(self.queue) and len(self.active) < self.max_slots:
            req = self.queue[i]
            nb = self.need(req)
            if nb > self.budget:
                del self.queue[i]
                self.rejected.append(req.rid)
                continue
            if self.in_use + nb <= self.budget:
                del self.queue[i]
                self.active[req.rid] = nb
                self.in_use += nb
                self.peak = max(self.peak, self.in_use)
                out.append(req)
                continue
            if skipped >= self.bypass:
                break
            skipped += 1
            i += 1
        return out

    def release(self, rid: int) -> None:
        self.in_use -= self.active.pop(rid)

    def idle(self) -> bool:
        return not self.queue and not self.active


# ---------------------------------------------------------------- GPU executor

@dataclasses.dataclass
class _Slot:
    req: Request
    plan: object
    stream: object
    x: object
    y: object
    r: object
    sens: object
    admitted: float
    enqueued: int = 0                          # EM iterations enqueued
    events: Deque = dataclasses.field(default_factory=collections.deque)
    host: object = None
    finishing: bool = False


class RequestData:
    """Host-side inputs of a request, generated from its seed: attenuation
    map, PSFs, Poisson sinogram y ~ Poisson(A x_true + r) with a uniform
    background r of 5% of the mean projection.  A x_true is computed with the
    GPU projector once, before the trace starts (the request arrives with its
    measured data).  The inputs are kept in pinned host memory, so that
    admitting the request copies them to the device asynchronously on its
    own stream; ``symmetric_x`` and ``symmetric_z`` record whether every PSF
    equals its mirror image in x and in z (checked here, on the host), which
    lets the plan pair taps without a device check (direct) or keep real
    spectra (FFT); ``request_bytes`` counts the complex spectra, an upper
    bound."""

    _psf_cache: Dict[str, np.ndarray] = {}

    def __init__(self, req: Request, device):
        import torch
        c = synth.CONFIGS[req.size]
        x, mu = synth.body_phantom(c["nx"], c["ny"], c["nz"], seed=req.seed)
        if req.size not in RequestData._psf_cache:   # the PSF model depends on the size only
            RequestData._psf_cache[req.size] = synth.gaussian_psf(
                c["px"], c["pz"], c["ny"], c["nview"], c["sigma"][0], c["sigma"][1])
        psf, dy = RequestData._psf_cache[req.size], c["dy"]
        self.x_true = x
        self.mu, self.psf, self.dy = mu, psf, dy
        plan = spect.Plan(torch.from_numpy(mu).to(device), torch.from_numpy(psf).to(device), dy)
        yc = plan.forward(torch.from_numpy(x).to(device))
        r = torch.full_like(yc, 0.05 * float(yc.mean()))
        gen = torch.Generator(device=device).manual_seed(req.seed)
        y = torch.poisson((yc + r).clamp_min(0.0), generator=gen)
        torch.cuda.synchronize(device)
        self.y = y.cpu().numpy()
        self.r = r.cpu().numpy()
        plan.close()
        self.symmetric_x = bool(np.array_equal(psf, psf[..., ::-1]))
        self.symmetric_z = bool(np.array_equal(psf, psf[..., ::-1, :]))
        self.pinned = {k: torch.from_numpy(getattr(self, k)).pin_memory()
                       for k in ("mu", "psf", "y", "r")}


class GpuExecutor:
    """Runs admitted requests on libspect: one plan (own workspace) per
    request, on one of ``max_slots`` streams created up front (default
    priority, reused so that the caching allocator recycles their memory).
    At most ``depth`` EM iterations of a request are in flight at once, so
    requests that share a hardware queue interleave at iteration
    granularity."""

    def __init__(self, device, data: Dict[int, RequestData], max_slots: int, depth: int = 2,
                 keep_results: bool = True, cache_mubar: bool = True):
        import torch
        self.torch = torch
        self.device = device
        self.data = data
        self.depth = depth
        self.keep = keep_results
        self.cache_mubar = cache_mubar
        self.free_streams = [torch.cuda.Stream(device=device) for _ in range(max_slots)]
        self.slots: Dict[int, _Slot] = {}

    def start(self, req: Request, now: float) -> None:
        """Admit a request without waiting on the device: its inputs are copied
        from pinned host memory on its own stream, the plan is created on that
        stream (with the PSF symmetry known from the host, so the plan does
        not wait for a device check), and the sensitivity back projection is
        enqueued behind them."""
        torch = self.torch
        d = self.data[req.rid]
        stream = self.free_streams.pop()
        with torch.cuda.stream(stream):
            mu, psf, y, r = (d.pinned[k].to(self.device, non_blocking=True)
                             for k in ("mu", "psf", "y", "r"))
            plan = spect.Plan(mu, psf, d.dy, cache_mubar=self.cache_mubar, precision=req.precision,
                              mirror="assume" if d.symmetric_x else "off", method=req.method,
                              symmetric_z=d.symmetric_z)
            sens = plan.back(torch.ones(plan.proj_shape, dtype=torch.float32, device=self.device))
            x = torch.ones(plan.vol_shape, dtype=torch.float32, device=self.device)
        self.slots[req.rid] = _Slot(req, plan, stream, x, y, r, sens, now)

    def step(self) -> None:
        """Top up every request to ``depth`` iterations in flight; after the
        last one, enqueue the copy of the image to pinned host memory."""
        torch = self.torch
        for s in self.slots.values():
            while s.events and s.events[0].query():
                s.events.popleft()
            while not s.finishing and len(s.events) < self.depth:
                with torch.cuda.stream(s.stream):
                    if s.enqueued < s.req.iters:
                        s.plan.em_step(s.x, s.y, s.sens, s.r)
                        s.enqueued += 1
                    else:
                        s.host = torch.empty(s.x.shape, dtype=torch.float32, pin_memory=True)
                        s.host.copy_(s.x, non_blocking=True)
                        s.finishing = True
                    ev = torch.cuda.Event()
                    ev.record(s.stream)
                    s.events.append(ev)

    def finished(self, now: float) -> List[Done]:
        out = []
        for rid in list(self.slots):
            s = self.slots[rid]
            if s.finishing and all(e.query() for e in s.events):
                x = s.host.numpy().copy() if self.keep else None
                out.append(Done(rid, s.req.size, s.req.arrival, s.admitted, now, x))
                s.plan.close()
                self.free_streams.append(s.stream)
                del self.slots[rid]
        return out


def serve(trace: List[Request], sched: Scheduler, executor, clock=time.perf_counter,
          poll_s: float = 2e-4) -> List[Done]:
    """Drive an arrival trace through the scheduler and executor: requests
    join the queue at their arrival time, are admitted as slots and memory
    free up, and progress an iteration at a time until every one is done."""
    pending = sorted(trace, key=lambda r: r.arrival)
    t0 = clock()
    done: List[Done] = []
    i = 0
    while i < len(pending) or not sched.idle():
        now = clock() - t0
        while i < len(pending) and pending[i].arrival <= now:
            sched.arrive(pending[i])
            i += 1
        for req in sched.admit():
            executor.start(req, now)
        executor.step()
        for d in executor.finished(clock() - t0):
            sched.release(d.rid)
            done.append(d)
        for rid in sched.rejected:
            if all(d.rid != rid for d in done):
                done.append(Done(rid, "rejected", float("nan"), float("nan"), float("nan")))
        sched.rejected.clear()
        if i < len(pending) and sched.idle():
            wait = pending[i].arrival - (clock() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.01))
        else:
            time.sleep(poll_s)
    return done


def summarize(done: List[Done], wall_s: float) -> dict:
    ok = [d for d in done if d.size != "rejected"]
    lat = sorted(d.latency for d in ok)

    def pct(q):
        if not lat:
            return None
        k = (len(lat) - 1) * q / 100.0
        lo = int(k)
        hi = min(lo + 1, len(lat) - 1)
        return (lat[lo] + (lat[hi] - lat[lo]) * (k - lo)) * 1e3

    by = collections.Counter(d.size for d in ok)
    return {"requests": len(ok), "rejected": len(done) - len(ok),
            "p50_ms": pct(50), "p99_ms": pct(99), "mean_ms": (1e3 * sum(lat) / len(lat)) if lat else None,
            "throughput_req_s": len(ok) / wall_s if wall_s > 0 else None,
            "by_size": dict(by)}
