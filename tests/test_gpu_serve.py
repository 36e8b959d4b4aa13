"""Continuous-batching EM service on the GPU: every request's result is the
same alone and in the mix (the kernels are deterministic and requests share
nothing but the device, so the bar is bitwise equality), equals a plain
em_step loop, and the memory budget holds under admission pressure."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2301_09710_amd import serve as sv  # noqa: E402
from paper_2301_09710_amd import spect  # noqa: E402

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mix():
    trace = [sv.Request(0, "serve64", 11, 0.000, iters=4),
             sv.Request(1, "serve96", 12, 0.002, iters=3),
             sv.Request(2, "serve64", 13, 0.004, iters=5),
             sv.Request(3, "paper", 14, 0.006, iters=2),
             sv.Request(4, "serve64", 15, 0.008, iters=4, precision="bf16"),
             sv.Request(5, "serve64", 16, 0.010, iters=3, method="fft"),
             sv.Request(6, "serve96", 17, 0.012, iters=2, method="fft")]
    say("serve: generating request data")
    data = {r.rid: sv.RequestData(r, DEV) for r in trace}
    return trace, data


def _run(trace, data, slots, budget):
    sched = sv.Scheduler(budget, slots,
                         lambda r: sv.request_bytes(r.size, r.precision, method=r.method))
    ex = sv.GpuExecutor(DEV, data, max_slots=slots)
    done = sv.serve(trace, sched, ex)
    torch.cuda.synchronize()
    return {d.rid: d for d in done}, sched


def test_results_same_alone_and_in_mix(mix):
    trace, data = mix
    say("serve: the mix, 4 slots")
    together, sched = _run(trace, data, 4, 64 << 30)
    assert sorted(together) == [r.rid for r in trace]
    for r in trace:
        say(f"serve: request {r.rid} alone")
        alone, _ = _run([sv.Request(r.rid, r.size, r.seed, 0.0, r.iters, r.precision, r.method)],
                        data, 1, 64 << 30)
        np.testing.assert_array_equal(alone[r.rid].x, together[r.rid].x)


def test_served_result_equals_plain_em_loop(mix):
    trace, data = mix
    r = trace[1]
    d = data[r.rid]
    plan = spect.Plan(torch.from_numpy(d.mu).to(DEV), torch.from_numpy(d.psf).to(DEV), d.dy,
                      cache_mubar=True)
    assert d.symmetric_x                       # the served plan pairs taps on the host's word
    sens = plan.back(torch.ones(plan.proj_shape, device=DEV))
    x = torch.ones(plan.vol_shape, device=DEV)
    y, rr = torch.from_numpy(d.y).to(DEV), torch.from_numpy(d.r).to(DEV)
    for _ in range(r.iters):
        plan.em_step(x, y, sens, rr)
    torch.cuda.synchronize()
    served, _ = _run([r], data, 1, 64 << 30)
    np.testing.assert_array_equal(served[r.rid].x, x.cpu().numpy())


def test_memory_budget_respected_under_pressure(mix):
    """The budget holds for the device memory the requests actually hold, as
    torch's allocator counts it (live buffers, already rounded to its 2 MiB
    granules), not only for the scheduler's own bookkeeping."""
    trace, data = mix
    need = {r.rid: sv.request_bytes(r.size, r.precision, method=r.method) for r in trace}
    budget = int(max(need.values()) * 1.2)          # the largest fits, never two large ones
    say(f"serve: budget {budget / 2 ** 30:.2f} GiB")
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated(DEV)
    torch.cuda.reset_peak_memory_stats(DEV)
    done, sched = _run(trace, data, 4, budget)
    measured = torch.cuda.max_memory_allocated(DEV) - base
    say(f"serve: admitted peak {sched.peak / 2 ** 30:.3f} GiB, measured peak "
        f"{measured / 2 ** 30:.3f} GiB")
    assert sorted(done) == [r.rid for r in trace]
    assert sched.peak <= budget
    assert measured <= budget


def test_request_bytes_counts_what_a_request_allocates(mix):
    """request_bytes is an upper bound on the device memory one admitted
    request allocates (measured around a served request alone)."""
    trace, data = mix
    for r in (trace[0], trace[3], trace[4], trace[6]):
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated(DEV)
        torch.cuda.reset_peak_memory_stats(DEV)
        _run([sv.Request(r.rid, r.size, r.seed, 0.0, r.iters, r.precision, r.method)], data, 1,
             64 << 30)
        measured = torch.cuda.max_memory_allocated(DEV) - base
        need = sv.request_bytes(r.size, r.precision, method=r.method)
        say(f"serve: {r.size}/{r.precision}/{r.method}: measured {measured / 2 ** 20:.1f} MiB, "
            f"request_bytes {need / 2 ** 20:.1f} MiB")
        assert measured <= need
