"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances
  FP64: every element within 1e-12 of the oracle, relative to the largest
        magnitude of the compared field (the bar set for the FP64 path).
  FP32: every element within 2e-6 relative to the largest magnitude after
        one step (float rounding of ~100 operations on values of one
        magnitude: a few tens of units in the last place, 2^-24 = 6e-8).

LBE boxes store post-collision populations, so the GPU result of a step from
a post-collision field P is compared with collide(stream(P)) of the oracle.
"""
import numpy as np
import pytest

import oracle as O
import paper_1601_03815_amd as dhit
import synth

pytestmark = pytest.mark.gpu

Q = 19
TOL64 = 1e-12
TOL32 = 2e-6


def rel_err(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def oracle_one_step(f, method, nu, dt=0.5):
    if method == "dugks":
        return O.dugks_step(f, nu=nu, dt=dt)
    return O.collide(O.stream(f), method, nu)


METHOD_VARIANTS = [("bgk", {}), ("mrt", {}), ("dugks", {}), ("dugks", {"variant": dhit.VARIANT_TWO_PASS})]


def _vid(mv):
    m, o = mv
    return m + ("-twopass" if o else "")


@pytest.mark.parametrize("mv", METHOD_VARIANTS, ids=_vid)
@pytest.mark.parametrize("n", [4, 5, 8, 12, 17, 32])
def test_one_step_fp64_random_state(mv, n):
    """One step from an arbitrary non-equilibrium state: grids from the
    minimum size through odd and ragged sizes (n^3 not a multiple of the
    256-cell block) to several tiles."""
    method, over = mv
    nu = 0.01
    f0 = synth.random_populations(n, seed=1000 + n, amplitude=0.01)
    with dhit.Box(n, method, "fp64", nu, **over) as box:
        box.set_populations(f0)
        box.step(1)
        got = box.get_populations()
        _, _, sums = box.moments(want_fields=False)
        hist = box.sums_history(1)[0]
    ref = oracle_one_step(f0, method, nu)
    assert rel_err(got, ref) <= TOL64
    ref_sums = O.moments(ref)[2]
    scale = np.abs(f0).sum()
    assert np.abs(sums - ref_sums).max() <= TOL64 * scale
    assert np.abs(hist - ref_sums).max() <= TOL64 * scale


@pytest.mark.parametrize("mv", METHOD_VARIANTS, ids=_vid)
@pytest.mark.parametrize("n", [5, 16])
def test_one_step_fp32_random_state(mv, n):
    method, over = mv
    nu = 0.01
    f0 = synth.random_populations(n, seed=2000 + n, amplitude=0.01)
    f0 = f0.astype(np.float32).astype(np.float64)   # representable start state
    with dhit.Box(n, method, "fp32", nu, **over) as box:
        box.set_populations(f0)
        box.step(1)
        got = box.get_populations()
    ref = oracle_one_step(f0, method, nu)
    assert rel_err(got, ref) <= TOL32


@pytest.mark.parametrize("method", ["bgk", "mrt", "dugks"])
def test_non_default_parameters(method):
    """Other viscosity, rho0, DUGKS time step and MRT rates go through."""
    n, nu = 6, 0.037
    over = dict(rho0=1.3)
    mrt = None
    if method == "dugks":
        over["dt"] = 0.35
    if method == "mrt":
        over.update(s1=1.5, s2=1.1, s4=1.3, s10=1.2, s16=1.7, w_eps=3.0, w_epsj=-5.5, w_xx=-0.5)
    f0 = synth.random_populations(n, seed=77, amplitude=0.02)
    with dhit.Box(n, method, "fp64", nu, **over) as box:
        box.set_populations(f0)
        box.step(1)
        got = box.get_populations()
    if method == "dugks":
        ref = O.dugks_step(f0, nu=nu, dt=0.35, rho0=1.3)
    else:
        if method == "mrt":
            s = O.mrt_rates(nu, s1=1.5, s2=1.1, s4=1.3, s10=1.2, s16=1.7)
            mrt = dict(s=s, w_eps=3.0, w_epsj=-5.5, w_xx=-0.5)
        ref = O.collide(O.stream(f0), method, nu, rho0=1.3, mrt=mrt)
    assert rel_err(got, ref) <= TOL64


@pytest.mark.parametrize("method", ["bgk", "mrt", "dugks"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_init_velocity_field(method, precision):
    n = 8
    u = synth.dhit_field(n, seed=3, k0=2, u_rms=0.05)
    drho = synth.random_populations(1, seed=4)[0, 0, 0, 0] + 0.001 * np.sin(np.arange(n ** 3)).reshape(n, n, n)
    with dhit.Box(n, method, precision, 0.01) as box:
        box.init_velocity_field(u, drho)
        got = box.get_populations()
        d, j, _ = box.moments()
    if method == "mrt":
        ref = O.init_mrt_equilibrium(u, drho)
    else:
        ref = O.init_equilibrium(u, drho)
    tol = TOL64 if precision == "fp64" else TOL32
    assert rel_err(got, ref) <= tol
    assert rel_err(j, u) <= tol
    assert rel_err(d, drho) <= tol


def test_taylor_green_config_fp64():
    """Taylor-Green vortex, 32^3, U0 = 0.05, nu = 0.01: 200 BGK-LBE and
    MRT-LBE steps and 400 DUGKS steps of dt = 0.5 (the same time, t = 200);
    populations after the run and the global sums reduced at the end of
    every step against the oracle's."""
    n, nu = 32, 0.01
    u = synth.taylor_green(n, 0.05)
    for method, steps in (("bgk", 200), ("mrt", 200), ("dugks", 400)):
        with dhit.Box(n, method, "fp64", nu) as box:
            box.init_velocity_field(u)
            box.step(steps)
            got = box.get_populations()
            hist = box.sums_history(steps)
        if method == "dugks":
            cur = O.init_equilibrium(u)
        elif method == "mrt":
            cur = O.init_mrt_equilibrium(u)
        else:
            cur = O.init_equilibrium(u)
        ref_hist = []
        for _ in range(steps):
            if method == "dugks":
                cur = O.dugks_step(cur, nu=nu)
            else:
                cur = O.lbe_step(cur, method, nu)
            ref_hist.append(O.moments(cur)[2])
        ref_hist = np.array(ref_hist)
        ref = cur if method == "dugks" else O.collide(cur, method, nu)
        assert rel_err(got, ref) <= TOL64, method
        np.testing.assert_allclose(hist[:, 4], ref_hist[:, 4], rtol=TOL64, atol=0)
        scale = np.abs(got).sum()
        assert np.abs(hist[:, :4] - ref_hist[:, :4]).max() <= TOL64 * scale


@pytest.mark.parametrize("n", [5, 16, 32])
def test_energy_spectrum_parity(n):
    nu = 0.005
    u = synth.dhit_field(n, seed=9, k0=4 if n >= 16 else 2, u_rms=0.05)
    kmax = int(np.ceil(np.sqrt(3) * (n // 2))) + 1
    with dhit.Box(n, "bgk", "fp64", nu) as box:
        box.init_velocity_field(u)
        E, st = box.energy_spectrum(kmax)
    E_ref, st_ref = O.energy_spectrum(u, nu, kmax)
    assert np.abs(E - E_ref).max() <= TOL64 * E_ref.max()
    for k in ("K", "eps"):
        assert abs(st[k] / st_ref[k] - 1) <= TOL64, k
    for k in ("S", "F"):
        assert abs(st[k] - st_ref[k]) <= 1e-10 * max(1.0, abs(st_ref[k])), k


def test_energy_spectrum_taylor_green_closed_form():
    n, u0, nu = 32, 0.05, 0.01
    with dhit.Box(n, "dugks", "fp64", nu) as box:
        box.init_velocity_field(synth.taylor_green(n, u0))
        E, st = box.energy_spectrum(n // 2)
    assert abs(st["K"] / (u0 ** 2 / 8) - 1) < 1e-13
    assert abs(E[2] / (u0 ** 2 / 8) - 1) < 1e-13
    assert abs(st["F"] - 27 / 8) < 1e-10 and abs(st["S"]) < 1e-10


def _sample_cells(n, count, seed):
    """Random cells plus every corner and the middle of every face and edge
    (where the periodic wrap is exercised)."""
    rng = np.random.default_rng(seed)
    pts = set(int(c) for c in rng.integers(0, n ** 3, count))
    for z in (0, n // 2, n - 1):
        for y in (0, n // 2, n - 1):
            for x in (0, n // 2, n - 1):
                pts.add((z * n + y) * n + x)
    return np.array(sorted(pts), dtype=np.int64)


@pytest.mark.parametrize("method", ["bgk", "mrt", "dugks"])
@pytest.mark.parametrize("n", [128, 256])
def test_full_size_sampled_cells_fp64(method, n):
    """Full-size boxes (the DHIT and benchmark sizes), in the launch
    configuration the benchmark times: one step from a random state, checked
    on sampled cells that the oracle computes one by one."""
    nu = 0.005 if n == 128 else 0.0025
    print("full-size sampled: %s n=%d" % (method, n), flush=True)
    f0 = synth.random_populations(n, seed=5 + n, amplitude=0.01)
    with dhit.Box(n, method, "fp64", nu) as box:
        box.set_populations(f0)
        box.step(1)
        got = box.get_populations().reshape(Q, -1)
    cells = _sample_cells(n, 3000, seed=n)
    if method == "dugks":
        ref = O.dugks_cells(f0, cells, nu=nu)
    else:
        ref = O.lbe_pull_cells(f0, cells, method, nu)
    assert rel_err(got[:, cells].T, ref) <= TOL64


@pytest.mark.parametrize("method", ["mrt", "dugks"])
@pytest.mark.parametrize("n", [128, 256])
def test_full_size_sampled_cells_fp32(method, n):
    """The FP32 deviation-form kernels at the benchmark's sizes and launch
    configuration: one step from a random state (rounded to FP32 on both
    sides), checked on sampled cells against the oracle's per-cell update."""
    nu = 0.005 if n == 128 else 0.0025
    print("full-size sampled fp32: %s n=%d" % (method, n), flush=True)
    f0 = synth.random_populations(n, seed=7 + n, amplitude=0.01).astype(np.float32).astype(np.float64)
    with dhit.Box(n, method, "fp32", nu) as box:
        box.set_populations(f0)
        box.step(1)
        got = box.get_populations().reshape(Q, -1)
    cells = _sample_cells(n, 3000, seed=n + 1)
    if method == "dugks":
        ref = O.dugks_cells(f0, cells, nu=nu)
    else:
        ref = O.lbe_pull_cells(f0, cells, method, nu)
    assert rel_err(got[:, cells].T, ref) <= TOL32


def test_step_method_mismatch_and_validation():
    with dhit.Box(4, "dugks", "fp64", 0.01) as box:
        with pytest.raises(dhit.DhitError) as e:
            dhit.step_lbe(box.handle, 1)
        assert e.value.code == -4
    with dhit.Box(4, "bgk", "fp64", 0.01) as box:
        with pytest.raises(dhit.DhitError) as e:
            dhit.step_dugks(box.handle, 1)
        assert e.value.code == -4
        with pytest.raises(dhit.DhitError):
            box.sums_history(1)   # no steps yet


def test_nonfinite_is_reported():
    n = 6
    f0 = synth.random_populations(n, seed=1)
    f0[3, 1, 2, 3] = np.nan
    with dhit.Box(n, "bgk", "fp64", 0.01) as box:
        box.set_populations(f0)
        box.step(2)
        with pytest.raises(dhit.NonFiniteError):
            box.synchronize()
        with pytest.raises(dhit.NonFiniteError):
            box.moments()


def test_torch_buffers_and_view():
    import torch
    n = 8
    u = synth.taylor_green(n, 0.05)
    with dhit.Box(n, "bgk", "fp64", 0.01) as box:
        box.init_velocity_field(u)
        box.step(3)
        torch.cuda.synchronize()
        view = box.populations_tensor().cpu().numpy()
        np.testing.assert_array_equal(view.reshape(Q, n, n, n), box.get_populations())
    with dhit.Box(n, "bgk", "fp64", 0.01, torch_memory=False) as box:
        box.init_velocity_field(u)
        box.step(3)
        np.testing.assert_array_equal(box.get_populations(), view.reshape(Q, n, n, n))


@pytest.mark.parametrize("method", ["bgk", "mrt", "dugks"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_equals_single_boxes(method, precision):
    """Boxes stepped in one batched launch equal the same boxes stepped alone
    bit for bit: the batch runs the same per-cell (LBE) or work-list (DUGKS:
    a single box is a table of one entry) kernel, and the DUGKS march rounds
    alike whatever the z-chunk."""
    sizes = [8, 12, 5, 16]
    states = [synth.random_populations(n, seed=40 + i) for i, n in enumerate(sizes)]
    singles = []
    for n, f in zip(sizes, states):
        with dhit.Box(n, method, precision, 0.01) as b:
            b.set_populations(f)
            b.step(3)
            singles.append(b.get_populations())
    boxes = [dhit.Box(n, method, precision, 0.01) for n in sizes]
    try:
        for b, f in zip(boxes, states):
            b.set_populations(f)
        dhit.step_boxes(boxes, 3)
        for b, ref in zip(boxes, singles):
            np.testing.assert_array_equal(b.get_populations(), ref)
            assert b.steps == 3
    finally:
        for b in boxes:
            b.close()


@pytest.mark.parametrize("method", ["bgk", "mrt", "dugks"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_graph_replays_equal_single_boxes(method, precision):
    """An autotuned batch replays its captured 8-step graph three times,
    with eager work of the program (moments, population reads, another box's
    steps) and synchronisations between the replays; after every replay each
    box equals the same box stepped alone (with the tile width the tuner
    chose) bit for bit, and the global sums of every step agree within the
    FP64 bar (the z-chunk decides how the cell sums are grouped)."""
    sizes = [8, 12, 5, 16, 24]
    states = [synth.random_populations(n, seed=70 + i, amplitude=0.01) for i, n in enumerate(sizes)]
    boxes = [dhit.Box(n, method, precision, 0.01) for n in sizes]
    other = dhit.Box(6, method, precision, 0.01)
    ref_boxes = []
    try:
        for b, f in zip(boxes, states):
            b.set_populations(f)
        other.set_populations(synth.random_populations(6, seed=99))
        with dhit.Batch(boxes, autotune=True) as bt:
            info = bt.info()
            assert info["tuned"] and info["grid"] > 0 and info["graph_steps"] == 8
            over = {"tile_width": info["tile"]} if method == "dugks" else {}
            if method == "dugks":
                assert info["tile"] in (16, 32)
            ref_boxes = [dhit.Box(n, method, precision, 0.01, **over) for n in sizes]
            for rb, f in zip(ref_boxes, states):
                rb.set_populations(f)
            for replay in range(3):
                bt.step(8)
                for rb in ref_boxes:
                    rb.step(8)
                for rb, b in zip(ref_boxes, boxes):
                    np.testing.assert_array_equal(b.get_populations(), rb.get_populations())
                    assert b.steps == rb.steps == 8 * (replay + 1)
                    hb, hr = b.sums_history(8), rb.sums_history(8)
                    scale = max(np.abs(hr).max(), 1e-30)
                    assert np.abs(hb - hr).max() <= 1e-12 * scale
                # eager work between replays
                other.step(2)
                boxes[0].moments()
        # the batch is gone; the boxes keep working on their own
        for rb, b in zip(ref_boxes, boxes):
            b.step(3)
            rb.step(3)
            if method != "dugks" or info["tile"] == 32:
                np.testing.assert_array_equal(b.get_populations(), rb.get_populations())
            else:
                # b steps alone with the default tile width now, rb with the tuned one
                assert rel_err(b.get_populations(), rb.get_populations()) <= (TOL64 if precision == "fp64" else TOL32)
    finally:
        for b in ref_boxes + boxes + [other]:
            b.close()


@pytest.mark.parametrize("method", ["bgk", "mrt", "dugks"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_against_oracle(method, precision):
    """A batch of mixed sizes (5, 8, 12, 16, 24) from random states, against
    the oracle: after one batched step (untuned) and after one replay of the
    autotuned batch's captured 8-step graph.  FP64: the 1e-12 bar.  FP32:
    k steps within k times the one-step bound (each step adds at most one
    step's rounding, relative to the largest population, and the schemes
    do not amplify a perturbation of that size within a few steps)."""
    nu = 0.01
    sizes = [5, 8, 12, 16, 24]
    states = []
    for i, n in enumerate(sizes):
        f = synth.random_populations(n, seed=500 + i, amplitude=0.01)
        if precision == "fp32":
            f = f.astype(np.float32).astype(np.float64)
        states.append(f)
    boxes = [dhit.Box(n, method, precision, nu) for n in sizes]
    try:
        for b, f in zip(boxes, states):
            b.set_populations(f)
        dhit.step_boxes(boxes, 1)
        refs = [oracle_one_step(f, method, nu) for f in states]
        for n, b, ref in zip(sizes, boxes, refs):
            err = rel_err(b.get_populations(), ref)
            print("batch vs oracle, 1 step: %s %s n=%d err %.3e" % (method, precision, n, err), flush=True)
            assert err <= (TOL64 if precision == "fp64" else TOL32), n
        # eight more steps in one graph replay of the tuned batch
        with dhit.Batch(boxes, autotune=True) as bt:
            bt.step(8)
        for n, b, f in zip(sizes, boxes, states):
            if method == "dugks":
                ref = O.dugks_step(f, nu=nu, nsteps=9)
            else:
                cur = O.stream(f)      # pre-collision state of the first GPU step
                for _ in range(8):
                    cur = O.lbe_step(cur, method, nu)
                ref = O.collide(cur, method, nu)
            err = rel_err(b.get_populations(), ref)
            print("batch vs oracle, 9 steps: %s %s n=%d err %.3e" % (method, precision, n, err), flush=True)
            assert err <= (TOL64 if precision == "fp64" else 9 * TOL32), n
            assert b.steps == 9
    finally:
        for b in boxes:
            b.close()


@pytest.mark.parametrize("method", ["mrt", "dugks"])
def test_batch_update_in_place(method):
    """A batch re-formed in place (batch_update: a box leaves and is
    destroyed, two join, a larger set than before) keeps stepping every box
    exactly as the box alone would (bit for bit), also through graph
    replays after each update."""
    sizes = {"a": 8, "b": 12, "c": 16, "d": 5, "e": 24}
    states = {k: synth.random_populations(n, seed=600 + i) for i, (k, n) in enumerate(sizes.items())}
    boxes = {k: dhit.Box(n, method, "fp32", 0.01) for k, n in sizes.items()}
    refs = {k: dhit.Box(n, method, "fp32", 0.01) for k, n in sizes.items()}
    try:
        for k in sizes:
            boxes[k].set_populations(states[k])
            refs[k].set_populations(states[k])
        bt = dhit.Batch([boxes["a"], boxes["b"], boxes["c"]], autotune=False)
        bt.step(9)
        for k in "abc":
            refs[k].step(9)
        boxes["b"].close()
        refs["b"].close()
        bt.update([boxes["a"], boxes["c"], boxes["d"], boxes["e"]])
        bt.step(17)
        for k in "acde":
            refs[k].step(17)
        bt.update([boxes["e"]])
        bt.step(8)
        refs["e"].step(8)
        bt.close()
        for k in "acde":
            np.testing.assert_array_equal(boxes[k].get_populations(), refs[k].get_populations())
            assert boxes[k].steps == refs[k].steps
    finally:
        for b in list(boxes.values()) + list(refs.values()):
            b.close()


def test_batch_rejects_mixed_boxes():
    a = dhit.Box(8, "bgk", "fp32", 0.01)
    b = dhit.Box(8, "dugks", "fp32", 0.01)
    try:
        with pytest.raises(dhit.DhitError):
            dhit.Batch([a, b])
        with pytest.raises(dhit.DhitError):
            dhit.Batch([a, a])
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("tile,chunk", [(16, 0), (32, 0), (16, 5), (32, 7), (16, 1), (32, -5)])
def test_dugks_tile_and_chunk_settings(precision, tile, chunk):
    """Every tile width and z-chunk (including chunks that do not divide n
    and single-plane chunks) gives the same step."""
    n, nu = 17, 0.01
    f0 = synth.random_populations(n, seed=300 + tile + chunk, amplitude=0.01)
    if precision == "fp32":
        f0 = f0.astype(np.float32).astype(np.float64)
    with dhit.Box(n, "dugks", precision, nu, tile_width=tile, z_chunk=chunk) as box:
        box.set_populations(f0)
        box.step(2)
        got = box.get_populations()
    ref = O.dugks_step(f0, nu=nu, nsteps=2)
    assert rel_err(got, ref) <= (TOL64 if precision == "fp64" else 2 * TOL32)


@pytest.mark.parametrize("precision,chunks", [("fp64", (7, -7, -2)), ("fp32", (3, -3, -2))])
def test_dugks_cut_last_round(precision, chunks):
    """A negative z_chunk launches the chunks on as many blocks as the device
    holds and cuts each chunk of a last, at most half full round into parts.
    At 64^3 with 32-wide tiles (33 column tiles) on a device of 256 compute
    units: FP64 (one block per unit) 7-plane chunks leave 74 chunks after one
    full round, cut into parts of 3, 3 and 1 planes (the last chunk, one
    plane, into 1, 0 and 0); 2-plane chunks leave 32 after four rounds; FP32
    (two blocks per unit) 3-plane chunks leave 214 after one round, cut in
    two.  Each split gives the oracle's two steps, the same populations as
    the uncut chunk bit for bit, and global sums equal to rounding."""
    n, nu = 64, 0.01
    f0 = synth.random_populations(n, seed=78, amplitude=0.01)
    if precision == "fp32":
        f0 = f0.astype(np.float32).astype(np.float64)
    ref = O.dugks_step(f0, nu=nu, nsteps=2)
    pops, hists = [], []
    for chunk in chunks:
        with dhit.Box(n, "dugks", precision, nu, tile_width=32, z_chunk=chunk) as box:
            box.set_populations(f0)
            box.step(2)
            pops.append(box.get_populations())
            hists.append(box.sums_history(2))
    assert rel_err(pops[0], ref) <= (TOL64 if precision == "fp64" else 2 * TOL32)
    for p, h in zip(pops[1:], hists[1:]):
        np.testing.assert_array_equal(p, pops[0])
        np.testing.assert_allclose(h, hists[0], rtol=0, atol=1e-12 * np.abs(f0).sum())


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_wide_reduction_equals_stored_state(precision):
    """At 192^3 the per-step reduction has more block partials than one
    block finalises (the wide finalisation runs, several blocks and an
    agent-scope counter); over three steps (the counter must come back to
    zero after each) the history sums and moments() equal the FP64 sums of
    the stored populations, computed here on the host.  FP64: to 1e-13 of
    sum |f|.  FP32: the LBE step sums the cells' compensated FP32 moments
    (taken before the collision, which conserves them), so the per-step sums
    differ from the stored values' by the FP32 rounding of each cell's
    moments (moments() forms them the same way): within 1e-7 of sum |f|
    (one rounding of 6e-8 per cell at most, accumulated linearly) and 1e-6
    of the energy; a block left out would be off by its share of the sum."""
    n = 192
    c, _ = O.lattice()
    f0 = synth.random_populations(n, seed=9, amplitude=0.01)
    if precision == "fp32":
        f0 = f0.astype(np.float32).astype(np.float64)
    with dhit.Box(n, "mrt", precision, 0.01) as b:
        b.set_populations(f0)
        for _ in range(3):
            b.step(1)
            f = b.get_populations()
            d = f.sum(axis=0)
            j = np.einsum("qa,q...->a...", c.astype(np.float64), f)
            ref = np.array([d.sum(), j[0].sum(), j[1].sum(), j[2].sum(), 0.5 * (j * j).sum()])
            scale = np.abs(f).sum()
            tol, etol = (1e-13, 1e-12) if precision == "fp64" else (1e-7, 1e-6)
            hist = b.sums_history(1)[0]
            mom = b.moments(want_fields=False)[2]
            for got in (hist, mom):
                assert np.abs(got[:4] - ref[:4]).max() <= tol * scale
                assert abs(got[4] / ref[4] - 1) <= etol
