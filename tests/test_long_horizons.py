"""Long parity and precision horizons against the oracle (minutes each; they
run only with DHIT_LONG=1 in the environment, and write their records as
JSON into the directory DHIT_LONG_OUT names, if set).

Decaying turbulence is chaotic: a difference of one rounding grows by orders
of magnitude within a few Kolmogorov times, so the GPU and the oracle cannot
agree element by element for ever.  These tests measure how long they do.

1. FP64 parity horizon at 128^3 (the 128^3 DHIT configuration: nu = 0.005,
   k0 = 4, u' = 0.05, seed 1): the library's box on the GPU and the oracle advance the same
   initial state in lockstep; every `every` steps the populations are
   compared element by element (largest |GPU - oracle| over the largest
   |oracle|).  The horizon is the first comparison above the 1e-12 bar; the
   first comparison must be within it.  Spans: 1500 MRT-LBE steps and 300
   DUGKS steps, or DHIT_LONG_MRT_STEPS / DHIT_LONG_DUGKS_STEPS (the whole
   three-turnover-time run is 6000 MRT-LBE steps); MRT-LBE comparisons every
   50 steps, or DHIT_LONG_MRT_EVERY.

2. FP32 against the FP64 oracle at 64^3 (the reduced-size check of the
   precision configuration: nu = 0.01, k0 = 4, u' = 0.05, seed 1) over three
   large-eddy turnover times t0 = K0/eps0 (Sec. IV.A): at every output (100
   LBE time units) the FP32 energy spectrum is compared with the oracle's
   shell by shell over the resolved shells (kappa_max eta <= 1 with the
   oracle's eta, shells holding at least 1e-10 of the largest), and K and
   eps; the error must stay within 1e-4 up to t0, and its horizon (first
   output above 1e-4) is recorded.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import paper_1601_03815_amd as dhit
import synth
from paper_1601_03815_amd.precision import resolved_shells

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not os.environ.get("DHIT_LONG"),
                                 reason="long measurement (minutes): set DHIT_LONG=1 to run it")]


def _save(name, rec):
    print(json.dumps(rec), flush=True)
    out = os.environ.get("DHIT_LONG_OUT")
    if out:
        os.makedirs(out, exist_ok=True)
        with open(os.path.join(out, name + ".json"), "w") as fh:
            json.dump(rec, fh, indent=1)


def _rel(got, ref):
    return float(np.abs(got - ref).max() / np.abs(ref).max())


@pytest.mark.parametrize("method,every,max_steps", [
    ("mrt", int(os.environ.get("DHIT_LONG_MRT_EVERY", "50")), int(os.environ.get("DHIT_LONG_MRT_STEPS", "1500"))),
    ("dugks", 25, int(os.environ.get("DHIT_LONG_DUGKS_STEPS", "300")))])
def test_fp64_parity_horizon_128(method, every, max_steps):
    n, nu = 128, 0.005
    u = synth.dhit_field(n, seed=1, k0=4, u_rms=0.05)
    cur = O.init_equilibrium(u) if method == "dugks" else O.init_mrt_equilibrium(u)
    rows, horizon = [], None
    with dhit.Box(n, method, "fp64", nu) as box:
        box.init_velocity_field(u)
        done = 0
        while done < max_steps:
            box.step(every)
            if method == "dugks":
                cur = O.dugks_step(cur, nu=nu, nsteps=every)
                ref = cur
            else:
                cur = O.lbe_step(cur, method, nu, nsteps=every)
                ref = O.collide(cur, method, nu)    # the GPU stores the post-collision phase
            done += every
            err = _rel(box.get_populations(), ref)
            rows.append((done, err))
            print("horizon 128^3 %s: step %d  max rel diff %.3e" % (method, done, err), flush=True)
            if horizon is None and err > 1e-12:
                horizon = done
            if horizon is not None and done >= horizon + 2 * every:
                break
    rec = {"case": "fp64 GPU vs oracle, 128^3 DHIT, nu=0.005, k0=4, u'=0.05, seed 1", "method": method,
           "every": every, "horizon_1e-12": horizon, "measured_steps": rows[-1][0],
           "rows": [dict(step=s, max_rel_diff=e) for s, e in rows]}
    _save("horizon_fp64_128_%s" % method, rec)
    assert rows[0][1] <= 1e-12


@pytest.mark.parametrize("method", ["mrt", "dugks"])
def test_fp32_against_oracle_64(method):
    n, nu, every = 64, 0.01, 100
    per = 2 if method == "dugks" else 1
    u = synth.dhit_field(n, seed=1, k0=4, u_rms=0.05)
    E0, st0 = O.energy_spectrum(u, nu, n // 2)
    t0 = st0["K"] / st0["eps"]
    outputs = int(math.ceil(3.0 * t0 / every))
    cur = O.init_equilibrium(u) if method == "dugks" else O.init_mrt_equilibrium(u)
    rows, horizon = [], None
    with dhit.Box(n, method, "fp32", nu) as box:
        box.init_velocity_field(u)
        for i in range(outputs + 1):
            if i:
                box.step(every * per)
                if method == "dugks":
                    cur = O.dugks_step(cur, nu=nu, nsteps=every * per)
                else:
                    cur = O.lbe_step(cur, method, nu, nsteps=every)
            E32, s32 = box.energy_spectrum(n // 2)
            _, j, _ = O.moments(cur)
            E64, s64 = O.energy_spectrum(j, nu, n // 2)
            kr = resolved_shells(n, nu, s64["eps"])
            ks = np.arange(1, kr + 1)
            ks = ks[E64[ks] >= 1e-10 * E64.max()]
            shell = float((np.abs(E32[ks] - E64[ks]) / E64[ks]).max())
            row = dict(t=i * every, t_over_t0=i * every / t0, shells=int(ks.max()), max_shell_rel=shell,
                       K_rel=float(abs(s32["K"] / s64["K"] - 1)), eps_rel=float(abs(s32["eps"] / s64["eps"] - 1)))
            rows.append(row)
            print("fp32 vs oracle 64^3 %s: t = %d (%.2f t0)  shell %.2e  K %.2e  eps %.2e"
                  % (method, row["t"], row["t_over_t0"], shell, row["K_rel"], row["eps_rel"]), flush=True)
            if horizon is None and shell > 1e-4:
                horizon = row["t"]
    rec = {"case": "fp32 GPU vs fp64 oracle, 64^3 DHIT, nu=0.01, k0=4, u'=0.05, seed 1", "method": method,
           "t0": t0, "horizon_1e-4": horizon, "rows": rows}
    _save("fp32_vs_oracle_64_%s" % method, rec)
    for row in rows:
        if row["t"] <= t0:
            assert row["max_shell_rel"] <= 1e-4, row
