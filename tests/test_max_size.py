"""The largest boxes one MI355X holds, where a population array passes 4 GiB
and the kernels address it with 64-bit offsets (FP32 n = 1024: 4 GiB per
population; FP64 n = 816: 4.3 GB), checked on every cell.

The oracle cannot hold such a box on the host, so the test uses a property
that holds at any size: the update is the same at every cell (Sec. II.A and
II.B: the scheme is translation invariant on the periodic grid), so a state
that repeats with period 16 along each axis stays periodic, and one step of
it equals, cell by cell, the oracle's step of the 16^3 periodic box it
repeats.  The repeated state is written into the box's device buffer with
PyTorch, the box steps once, and the result is compared with the tiled
16^3 oracle result on the GPU, one population at a time.  The per-step
global sums (FP64) must equal 64^3 (or 51^3) times the 16^3 box's.
"""
import numpy as np
import pytest

import oracle as O
import synth

P = 16
TOL64, TOL32 = 1e-12, 2e-6


@pytest.mark.gpu
@pytest.mark.parametrize("method,precision,n", [
    ("mrt", "fp32", 1024), ("dugks", "fp32", 1024),
    ("mrt", "fp64", 816), ("dugks", "fp64", 816)])
def test_largest_boxes_every_cell(method, precision, n):
    import torch

    import paper_1601_03815_amd as dhit
    assert n % P == 0
    nu = 0.0025
    print("max size: %s %s n=%d" % (method, precision, n), flush=True)
    f16 = synth.random_populations(P, seed=n + len(method), amplitude=0.01)
    if precision == "fp32":
        f16 = f16.astype(np.float32).astype(np.float64)
    if method == "dugks":
        ref16 = O.dugks_step(f16, nu=nu)
    else:
        ref16 = O.lbe_pull_cells(f16, np.arange(P ** 3), method, nu).T.reshape(19, P, P, P)
    _, _, sums16 = O.moments(ref16)
    dt = torch.float64 if precision == "fp64" else torch.float32
    reps = n // P
    torch.cuda.empty_cache()   # the box takes 150-170 GB: return what earlier tests cached
    box = dhit.Box(n, method, precision, nu)
    try:
        cur = box.populations_tensor()
        with torch.cuda.stream(box.stream):
            for q in range(19):
                tile = torch.from_numpy(f16[q]).to(device="cuda", dtype=dt)
                cur[q].view(n, n, n).copy_(tile.repeat(reps, reps, reps))
        box.stream.synchronize()
        box.step(1)
        got = box.populations_tensor()   # waits for the step
        sums = box.sums_history(1)[0]
        scale = float(np.abs(ref16).max())
        worst = 0.0
        with torch.cuda.stream(box.stream):
            for q in range(19):
                r = torch.from_numpy(ref16[q]).to(device="cuda", dtype=torch.float64)
                g = got[q].view(reps, P, reps, P, reps, P)
                d = (g.to(torch.float64) - r[None, :, None, :, None, :]).abs().max()
                worst = max(worst, float(d))
        box.stream.synchronize()
    finally:
        box.close()
        torch.cuda.empty_cache()
    tol = TOL64 if precision == "fp64" else TOL32
    print("max size: %s %s n=%d: largest |GPU - oracle| / max|oracle| = %.3e" % (method, precision, n, worst / scale),
          flush=True)
    assert worst <= tol * scale
    # sums over the whole box: reps^3 copies of the 16^3 box's sums
    ref_sums = sums16 * reps ** 3
    sum_scale = np.abs(ref16).sum() * reps ** 3
    assert np.abs(sums - ref_sums).max() <= (1e-12 if precision == "fp64" else 1e-6) * sum_scale


@pytest.mark.parametrize("method", ["bgk", "mrt", "dugks"])
def test_periodic_tiling_premise_on_the_oracle(method):
    """The premise, on the CPU with the oracle alone: one step of a 4^3
    state repeated twice along each axis equals the repeated step of the
    4^3 box, and the reference is assembled in the cell order the test
    uses."""
    nu, p, reps = 0.0025, 4, 2
    f4 = synth.random_populations(p, seed=3, amplitude=0.01)
    f8 = np.tile(f4, (1, reps, reps, reps))
    if method == "dugks":
        r4, r8 = O.dugks_step(f4, nu=nu), O.dugks_step(f8, nu=nu)
    else:
        r4 = O.lbe_pull_cells(f4, np.arange(p ** 3), method, nu).T.reshape(19, p, p, p)
        r8 = O.lbe_pull_cells(f8, np.arange((p * reps) ** 3), method, nu).T.reshape(19, p * reps, p * reps, p * reps)
    assert np.abs(r8 - np.tile(r4, (1, reps, reps, reps))).max() <= 1e-16
    _, _, s4 = O.moments(r4)
    _, _, s8 = O.moments(r8)
    assert np.abs(s8 - reps ** 3 * s4).max() <= 1e-14 * np.abs(r8).sum()
