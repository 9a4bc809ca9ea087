"""Serving loop: scheduler logic on the CPU with a fake backend, and on the
GPU the requirement that each result is the same alone and in the mix."""
import numpy as np
import pytest

from paper_1601_03815_amd.serve import Request, Scheduler, poisson_trace


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(0.0, dt)


class FakeBackend:
    """Simulated device: a run of n^3 cells costs n^3 * steps / rate seconds
    of device time; memory is 2 * 8 * 19 * n^3 bytes."""

    def __init__(self, clock, rate=1e9):
        self.clock, self.rate = clock, rate
        self.live = {}
        self.steps = {}
        self.order = []

    def bytes_of(self, req):
        return 2 * 8 * 19 * req.n ** 3

    def start(self, req):
        self.live[req.rid] = req
        self.steps[req.rid] = 0
        self.order.append(req.rid)
        return req.rid

    def advance(self, handles, nsteps):
        cost = sum(self.live[h].n ** 3 for h in handles) * nsteps / self.rate
        self.clock.t += cost
        for h in handles:
            self.steps[h] += nsteps

    def finish(self, h):
        return {"steps": self.steps[h]}

    def release(self, h):
        del self.live[h]

    def sync(self):
        pass


def test_trace_is_seeded_and_shaped():
    a = poisson_trace(200, 20.0, seed=3)
    b = poisson_trace(200, 20.0, seed=3)
    assert [(r.arrival, r.n, r.method, r.steps) for r in a] == [(r.arrival, r.n, r.method, r.steps) for r in b]
    assert all(x.arrival < y.arrival for x, y in zip(a, a[1:]))
    assert {r.n for r in a} <= {32, 64, 128, 256} and {r.method for r in a} == {"mrt", "dugks"}
    assert all(500 <= r.steps <= 2000 for r in a)
    gaps = np.diff([0.0] + [r.arrival for r in a])
    assert 0.03 < gaps.mean() < 0.07            # mean 1/20 s


@pytest.mark.parametrize("budget_gb,max_active", [(1000.0, 64), (16.0, 64), (16.0, 3)])
def test_scheduler_budget_order_and_completion(budget_gb, max_active):
    clock = FakeClock()
    be = FakeBackend(clock)
    trace = poisson_trace(60, 20.0, seed=5)
    sch = Scheduler(be, budget_gb * 1e9, max_active=max_active, chunk=64)
    stats = sch.run(trace, clock=clock, sleep=clock.sleep)
    assert stats["requests"] == 60
    assert sch.peak_in_use <= budget_gb * 1e9
    assert not be.live and sch.in_use == 0
    for r in trace:                              # every run got exactly its steps
        res = sch.results[r.rid]
        assert res["result"]["steps"] == r.steps
        assert res["latency"] >= r.n ** 3 * r.steps / be.rate - 1e-9
        assert res["wait"] >= 0
    assert be.order == sorted(be.order)          # admitted first come, first served
    assert stats["p99_s"] >= stats["p50_s"] > 0


def test_scheduler_admits_while_others_run():
    """A request arriving while a long run is active starts before that run ends."""
    clock = FakeClock()
    be = FakeBackend(clock, rate=1e6)
    trace = [Request(0.0, 0, 64, "mrt", 2000, 1), Request(0.01, 1, 32, "dugks", 100, 2)]
    sch = Scheduler(be, 1e12, chunk=50)
    sch.run(trace, clock=clock, sleep=clock.sleep)
    assert sch.results[1]["latency"] < sch.results[0]["latency"]
    assert sch.results[1]["wait"] < 64 ** 3 * 2000 / be.rate


def test_scheduler_rejects_oversized_request():
    clock = FakeClock()
    sch = Scheduler(FakeBackend(clock), 1e6)
    with pytest.raises(ValueError):
        sch.run([Request(0.0, 0, 64, "mrt", 10, 1)], clock=clock, sleep=clock.sleep)


def test_prepare_is_called_once_per_request_after_arrival_before_start():
    """A backend's prepare hook (initial-field generation ahead of admission)
    sees every request once, no earlier than its arrival and before start."""
    clock = FakeClock()

    class PreparingBackend(FakeBackend):
        def __init__(self, clock):
            super().__init__(clock, rate=1e6)
            self.prepared = {}

        def prepare(self, req):
            assert req.rid not in self.prepared
            assert clock() >= req.arrival
            self.prepared[req.rid] = clock()

        def start(self, req):
            assert req.rid in self.prepared
            return super().start(req)

    be = PreparingBackend(clock)
    trace = poisson_trace(30, 50.0, seed=5, grids=(16, 32), weights=(1, 1), steps=(50, 200))
    sch = Scheduler(be, 40 * 2 * 8 * 19 * 32 ** 3, max_active=4, chunk=25)
    sch.run(trace, clock=clock, sleep=clock.sleep)
    assert sorted(be.prepared) == sorted(r.rid for r in trace)
    assert len(sch.results) == len(trace)


@pytest.mark.gpu
def test_result_is_the_same_alone_and_in_the_mix():
    """Runs served together (continuous batching, both methods overlapping on
    two streams) give the same result as each run alone on its own box, bit
    for bit: the batched kernels equal the single-box ones bit for bit, and
    the spectrum's shell sums are exact integer sums.  A few served runs are
    also checked against the FP64 oracle (same initial field, same steps):
    the FP32 spectrum within 1e-4 of the oracle's at every shell holding at
    least 1e-10 of the largest, K within 1e-5."""
    import oracle as O
    import paper_1601_03815_amd as dhit
    import synth
    from paper_1601_03815_amd.serve import GpuBackend

    trace = poisson_trace(12, 200.0, seed=11, grids=(8, 12, 16), weights=(1, 1, 1), steps=(20, 60))
    be = GpuBackend(precision="fp32", nu=0.01)
    sch = Scheduler(be, 4e9, chunk=16)
    stats = sch.run(trace)
    be.close()
    assert stats["requests"] == len(trace)
    for r in trace:
        u = synth.dhit_field_gpu(r.n, seed=r.seed, k0=4.0, u_rms=0.05)   # the backend's field recipe
        with dhit.Box(r.n, r.method, "fp32", 0.01) as b:
            b.init_velocity_field(u)
            b.step(r.steps)
            E, st = b.energy_spectrum(r.n // 2)
        got = sch.results[r.rid]["result"]
        np.testing.assert_array_equal(got["E"], E)
        for k in ("K", "eps", "S", "F"):
            assert got[k] == st[k], (r.rid, k)
    # oracle checks of served runs: the first of each method and grid size
    checked = set()
    for r in trace:
        if (r.method, r.n) in checked:
            continue
        checked.add((r.method, r.n))
        u = synth.dhit_field(r.n, seed=r.seed, k0=4.0, u_rms=0.05)
        if r.method == "dugks":
            f = O.dugks_step(O.init_equilibrium(u), nu=0.01, nsteps=r.steps)
        else:
            f = O.lbe_step(O.init_mrt_equilibrium(u), r.method, 0.01, nsteps=r.steps)
        _, j, _ = O.moments(f)
        E_ref, st_ref = O.energy_spectrum(j, 0.01, r.n // 2)
        got = sch.results[r.rid]["result"]
        keep = E_ref >= 1e-10 * E_ref.max()
        keep[0] = False
        err = float((np.abs(got["E"] - E_ref)[keep] / E_ref[keep]).max())
        print("served vs oracle: %s n=%d steps=%d shell error %.2e" % (r.method, r.n, r.steps, err), flush=True)
        assert err <= 1e-4, (r.rid, err)
        assert abs(got["K"] / st_ref["K"] - 1) <= 1e-5
    assert len(checked) >= 4


@pytest.mark.gpu
@pytest.mark.parametrize("n", [32, 128])
def test_spectrum_bytes_covers_the_work_space(n):
    """spectrum_bytes (what the serving loop reserves for a run's final
    spectrum) covers what energy_spectrum actually allocates on the device:
    the arrays (3 velocity fields, 4 half spectra) and the hipFFT plans'
    work areas.  Device memory is read with hipMemGetInfo through PyTorch;
    allocations are rounded up to pages, hence the slack."""
    import torch

    import paper_1601_03815_amd as dhit
    import synth
    p = dhit.default_params(n, "mrt", "fp32", 0.01)
    need = dhit.spectrum_bytes(p)
    arrays = 3 * n ** 3 * 8 + 4 * n * n * (n // 2 + 1) * 16
    assert need >= arrays
    with dhit.Box(n, "mrt", "fp32", 0.01) as b:
        b.init_velocity_field(synth.taylor_green(n, 0.05))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        b.energy_spectrum()
        torch.cuda.synchronize()
        used = free0 - torch.cuda.mem_get_info()[0]
    print("n=%d spectrum_bytes %d, device memory taken %d" % (n, need, used), flush=True)
    assert used <= need + (64 << 20)


@pytest.mark.parametrize("n", [8, 16, 33])
def test_torch_field_recipe_matches_host_recipe(n):
    """synth.dhit_field_gpu (the recipe's transforms through PyTorch; run
    here on the CPU device) gives dhit_field's field to FFT rounding, and the
    same bits on every call."""
    import synth
    ref = synth.dhit_field(n, seed=5, k0=4.0, u_rms=0.05)
    got = synth.dhit_field_gpu(n, seed=5, k0=4.0, u_rms=0.05, device="cpu")
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    np.testing.assert_array_equal(got, synth.dhit_field_gpu(n, seed=5, k0=4.0, u_rms=0.05, device="cpu"))


@pytest.mark.gpu
def test_torch_field_recipe_on_the_gpu():
    import synth
    ref = synth.dhit_field(64, seed=6, k0=4.0, u_rms=0.05)
    got = synth.dhit_field_gpu(64, seed=6, k0=4.0, u_rms=0.05)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    np.testing.assert_array_equal(got, synth.dhit_field_gpu(64, seed=6, k0=4.0, u_rms=0.05))


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["bgk", "mrt", "dugks"])
def test_device_init_equals_host_init(method, precision):
    """init_velocity_field_device (fields already on the device, no staging,
    asynchronous on the box's stream) builds the same state as
    init_velocity_field, bit for bit, with and without drho, and the boxes
    step alike."""
    import torch

    import paper_1601_03815_amd as dhit
    import synth
    n = 13
    u = synth.dhit_field(n, seed=4, k0=2, u_rms=0.05)
    d = 1e-3 * synth.random_populations(n, seed=9)[0]
    for drho in (None, d):
        with dhit.Box(n, method, precision, 0.01) as a, dhit.Box(n, method, precision, 0.01) as b:
            a.init_velocity_field(u, drho)
            ud = torch.from_numpy(u).cuda()
            dd = None if drho is None else torch.from_numpy(drho).cuda()
            b.init_velocity_field_device(ud, dd)
            del ud, dd
            np.testing.assert_array_equal(a.get_populations(), b.get_populations())
            a.step(3)
            b.step(3)
            np.testing.assert_array_equal(a.get_populations(), b.get_populations())
            assert b.steps == 3


@pytest.mark.gpu
def test_pooled_boxes_give_the_same_result():
    """At most two runs at a time, so later runs take the boxes of earlier
    ones from the backend's pool: with one grid size and two methods at most
    four boxes of a method are busy at once (two running, two waiting to be
    finished), so 12 runs cannot need 12 boxes.  Every result equals the same
    run alone on a fresh box, bit for bit."""
    import paper_1601_03815_amd as dhit
    import synth
    from paper_1601_03815_amd.serve import GpuBackend

    trace = poisson_trace(12, 100.0, seed=21, grids=(12,), weights=(1,), steps=(20, 40))
    be = GpuBackend(precision="fp32", nu=0.01)
    sch = Scheduler(be, 4e9, max_active=2, chunk=8)
    stats = sch.run(trace)
    be.close()
    assert stats["requests"] == len(trace)
    assert be.created < len(trace), be.created
    for r in trace:
        u = synth.dhit_field_gpu(r.n, seed=r.seed, k0=4.0, u_rms=0.05)
        with dhit.Box(r.n, r.method, "fp32", 0.01) as b:
            b.init_velocity_field(u)
            b.step(r.steps)
            E, st = b.energy_spectrum(r.n // 2)
        got = sch.results[r.rid]["result"]
        np.testing.assert_array_equal(got["E"], E)
        for k in ("K", "eps", "S", "F"):
            assert got[k] == st[k], (r.rid, k)


@pytest.mark.gpu
@pytest.mark.parametrize("method", ["mrt", "dugks"])
def test_batch_on_a_stream_of_its_own(method):
    """A batch issued on a third stream (batch_set_stream) while each box
    keeps its own stream: the boxes' states after 9 steps (one graph replay
    and one eager step) and their spectra, computed on the boxes' streams
    right after the batch steps, equal the same boxes stepped alone."""
    import torch

    import paper_1601_03815_amd as dhit
    import synth
    sizes = (8, 12, 16)
    fields = [synth.dhit_field(n, seed=30 + n, k0=2, u_rms=0.05) for n in sizes]
    boxes = [dhit.Box(n, method, "fp32", 0.01, stream=torch.cuda.Stream()) for n in sizes]
    for b, u in zip(boxes, fields):
        b.init_velocity_field(u)
    bt = dhit.Batch(boxes, autotune=False, stream=torch.cuda.Stream())
    bt.step(9)
    got = [(b.energy_spectrum(), b.get_populations()) for b in boxes]
    bt.close()
    for b in boxes:
        b.close()
    for (E_st, f), n, u in zip(got, sizes, fields):
        with dhit.Box(n, method, "fp32", 0.01) as a:
            a.init_velocity_field(u)
            a.step(9)
            E, st = a.energy_spectrum()
            np.testing.assert_array_equal(f, a.get_populations())
        np.testing.assert_array_equal(E_st[0], E)
        assert E_st[1]["K"] == st["K"]


@pytest.mark.gpu
def test_device_init_and_batch_stream_errors():
    """Error paths of the two entry points the serving loop uses: a null
    velocity field, wrong tensor shapes or types, a null batch."""
    import torch

    import paper_1601_03815_amd as dhit
    from paper_1601_03815_amd import _binding
    with dhit.Box(6, "mrt", "fp64", 0.01) as b:
        with pytest.raises(dhit.DhitError) as e:
            dhit.init_velocity_field_device(b.handle, 0)
        assert e.value.code == -1
        with pytest.raises(ValueError):
            b.init_velocity_field_device(torch.zeros((3, 6, 6, 5), dtype=torch.float64, device="cuda"))
        with pytest.raises(ValueError):
            b.init_velocity_field_device(torch.zeros((3, 6, 6, 6), dtype=torch.float32, device="cuda"))
        with pytest.raises(ValueError):
            b.init_velocity_field_device(torch.zeros((3, 6, 6, 6), dtype=torch.float64))
    with pytest.raises(dhit.DhitError) as e:
        _binding.batch_set_stream(None, 0)
    assert e.value.code == -1


def test_prepare_may_decline_and_is_asked_again():
    """A backend that holds at most two prepared requests declines the rest
    (returns False); the scheduler asks again in later rounds, in arrival
    order, and every request is still prepared before it starts."""
    clock = FakeClock()

    class Bounded(FakeBackend):
        def __init__(self, clock):
            super().__init__(clock, rate=1e6)
            self.held, self.prepared, self.asked = set(), [], []

        def prepare(self, req):
            self.asked.append(req.rid)
            if len(self.held) >= 2:
                return False
            self.held.add(req.rid)
            self.prepared.append(req.rid)
            return True

        def start(self, req):
            assert req.rid in self.held
            self.held.discard(req.rid)
            return super().start(req)

    be = Bounded(clock)
    trace = poisson_trace(20, 100.0, seed=8, grids=(16, 32), weights=(1, 1), steps=(50, 200))
    sch = Scheduler(be, 1e12, max_active=2, chunk=25)
    sch.run(trace, clock=clock, sleep=clock.sleep)
    assert len(sch.results) == len(trace)
    assert be.prepared == sorted(be.prepared)          # prepared in arrival order
    assert sorted(be.prepared) == [r.rid for r in trace]
    assert len(be.asked) > len(trace)                  # some were declined and asked again
