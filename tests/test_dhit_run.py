"""The 128^3 decaying-turbulence configuration on the GPU: FP64, nu = 0.005,
DHIT field with k0 = 4, u' = 0.05, seed 1, run for three large-eddy
turnover times t0 = K0/eps0 of the initial field (Sec. IV.A), with E(k),
eps, S (and K, F) output every 100 LBE time units (every 100 MRT-LBE steps,
every 200 DUGKS steps of dt = 0.5).  The oracle cannot run this length, and
the flow is chaotic (its GPU-vs-oracle parity horizon is measured in
test_long_horizons.py), so the run is checked against properties of the
flow:
  * the collision and the flux form conserve sum drho and sum j (round-off);
  * K decays monotonically;
  * eps is positive, rises from the initial field to a peak as the energy
    cascade develops (Sec. IV.B) and then decays;
  * the velocity-derivative skewness of the developed flow is negative,
    between -0.6 and -0.3, and the flatness between 3 and 5;
  * the two methods give the same K(t) within 10% up to one turnover time;
    later the DUGKS, whose reconstruction damps the poorly resolved high
    wavenumbers, dissipates less and keeps more energy (Sec. IV.B and IV.C
    compare them).
"""
import math

import numpy as np
import pytest

import paper_1601_03815_amd as dhit
import synth

pytestmark = pytest.mark.gpu

N, NU, EVERY = 128, 0.005, 100   # outputs every 100 LBE time units


def _field():
    return synth.dhit_field(N, seed=1, k0=4, u_rms=0.05)


def _turnover_time(u):
    with dhit.Box(N, "mrt", "fp64", NU) as b:
        b.init_velocity_field(u)
        _, st = b.energy_spectrum()
    return st["K"] / st["eps"]


def _run(method, u, outputs):
    per = 2 if method == "dugks" else 1
    rows, sums = [], []
    with dhit.Box(N, method, "fp64", NU) as b:
        b.init_velocity_field(u)
        _, st = b.energy_spectrum()
        rows.append((0.0, st["K"], st["eps"], st["S"], st["F"]))
        for i in range(outputs):
            b.step(EVERY * per)
            sums.append(b.sums_history(EVERY * per))
            _, st = b.energy_spectrum()
            rows.append((EVERY * (i + 1), st["K"], st["eps"], st["S"], st["F"]))
    return np.array(rows), np.concatenate(sums)


@pytest.fixture(scope="module")
def runs():
    u = _field()
    t0 = _turnover_time(u)
    outputs = int(math.ceil(3.0 * t0 / EVERY))
    print("dhit 128^3: t0 = %.1f time units; mrt %d steps, dugks %d steps, %d outputs"
          % (t0, outputs * EVERY, 2 * outputs * EVERY, outputs), flush=True)
    out = {m: _run(m, u, outputs) for m in ("mrt", "dugks")}
    out["t0"] = t0
    return out


def test_runs_three_turnover_times(runs):
    rows, _ = runs["mrt"]
    assert rows[-1, 0] >= 3.0 * runs["t0"]
    assert np.all(np.diff(rows[:, 0]) == EVERY)


@pytest.mark.parametrize("method", ["mrt", "dugks"])
def test_conservation(runs, method):
    _, sums = runs[method]
    assert np.abs(sums[:, 0]).max() <= 1e-8
    assert np.abs(sums[:, 1:4]).max() <= 1e-8


@pytest.mark.parametrize("method", ["mrt", "dugks"])
def test_energy_decay_and_dissipation(runs, method):
    rows, sums = runs[method]
    K, eps = rows[:, 1], rows[:, 2]
    assert np.all(np.diff(K) < 0)
    assert np.all(eps > 0)
    peak = int(np.argmax(eps))
    assert 0 < peak < len(eps) - 1
    assert eps[peak] > 1.5 * eps[0] and eps[-1] < 0.5 * eps[peak]
    # the per-step kinetic-energy reduction agrees with the spectrum's K
    # (same field: 1/2 sum |u|^2 over the cells, the mean over them is K)
    assert abs(sums[-1, 4] / N ** 3 / K[-1] - 1) <= 1e-9


@pytest.mark.parametrize("method", ["mrt", "dugks"])
def test_developed_derivative_statistics(runs, method):
    rows, _ = runs[method]
    t0 = runs["t0"]
    dev = rows[:, 0] >= 0.4 * t0           # once the cascade has developed
    S, F = rows[dev, 3], rows[dev, 4]
    print("%s: S in [%.3f, %.3f], F in [%.3f, %.3f]" % (method, S.min(), S.max(), F.min(), F.max()), flush=True)
    assert np.all((S > -0.6) & (S < -0.3))
    assert np.all((F > 3.0) & (F < 5.0))


def test_methods_agree_on_energy_decay(runs):
    """The two methods give the same K(t) within 10% up to one turnover time.
    Later the DUGKS keeps more energy: its face reconstruction damps the
    high wavenumbers that this grid does not resolve well at Re_lambda ~ 100,
    so its resolved dissipation rate falls below the LBE's (Sec. IV.C finds
    the DUGKS's dissipation rate up to 27% off the reference at 128^3 and
    this Re_lambda, against 4.5% for the LBE, the differences showing
    around the dissipation peak): eps(DUGKS) is below eps(LBE) by more than
    2% at the LBE's dissipation peak, and K(DUGKS) > K(LBE), by no more than
    25%, after one turnover time."""
    rows_l, rows_d = runs["mrt"][0], runs["dugks"][0]
    t, K_l, K_d = rows_l[:, 0], rows_l[:, 1], rows_d[:, 1]
    e_l, e_d = rows_l[:, 2], rows_d[:, 2]
    r, re = K_d / K_l - 1, e_d / e_l - 1
    pick = [int(np.argmin(np.abs(t - f * runs["t0"]))) for f in (0.5, 1, 2, 3)]
    print("at t/t0 = 0.5, 1, 2, 3: K(dugks)/K(mrt) - 1 = %s; eps(dugks)/eps(mrt) - 1 = %s"
          % (", ".join("%.4f" % r[i] for i in pick), ", ".join("%.4f" % re[i] for i in pick)), flush=True)
    early = t <= runs["t0"]
    assert np.abs(r[early]).max() <= 0.10
    late = t > runs["t0"]
    assert np.all(r[late] > 0) and np.all(r[late] < 0.25)
    assert re[int(np.argmax(e_l))] < -0.02
