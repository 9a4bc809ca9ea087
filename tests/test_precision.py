"""FP32 deviation-form path against the FP64 path and the oracle over a
horizon (GPU)."""
import numpy as np
import pytest

import oracle as O
import paper_1601_03815_amd as dhit
import synth
from paper_1601_03815_amd.precision import compare_fp32_fp64, resolved_shells

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("method", ["mrt", "dugks"])
def test_fp32_spectrum_error_below_1e4_over_horizon(method):
    """DHIT 32^3, nu = 0.01, k0 = 4, u' = 0.05: the FP32 energy spectrum stays
    within 1e-4 of the FP64 one at every resolved shell for 200 LBE time
    units (200 LBE steps, 400 DUGKS steps), checked every 50 time units."""
    u = synth.dhit_field(32, seed=1, k0=4, u_rms=0.05)
    steps = 200 if method == "mrt" else 400
    out, horizon = compare_fp32_fp64(u, method, 0.01, steps, steps // 4, threshold=1e-4)
    assert horizon is None, out
    assert max(r["K_rel"] for r in out) < 1e-4
    assert max(r["eps_rel"] for r in out) < 1e-4


def test_fp32_dugks_energy_has_no_systematic_drift():
    """DHIT 32^3, nu = 0.01, 800 DUGKS steps: the FP32 kinetic energy stays
    within 4e-6 of the FP64 one.  An equilibrium whose linear coefficients
    carry the weights' FP32 rounding (momentum j (1 + 7e-9)) makes every DUGKS
    collision add a fixed fraction of it: K then drifts by ~3e-8 per step,
    2.6e-5 after 800 steps."""
    u = synth.dhit_field(32, seed=3, k0=4, u_rms=0.05)
    out, _ = compare_fp32_fp64(u, "dugks", 0.01, 800, 200, threshold=1e-4)
    assert max(r["K_rel"] for r in out) < 4e-6, out


@pytest.mark.parametrize("method", ["mrt", "dugks"])
def test_fp64_spectrum_matches_oracle_over_horizon(method):
    """DHIT 24^3: the FP64 GPU spectrum, K and eps match the oracle's at every
    resolved shell within 1e-12 after 60 LBE time units."""
    n, nu = 24, 0.01
    u = synth.dhit_field(n, seed=2, k0=4, u_rms=0.05)
    steps = 60 if method == "mrt" else 120
    with dhit.Box(n, method, "fp64", nu) as b:
        b.init_velocity_field(u)
        b.step(steps)
        E, st = b.energy_spectrum(n // 2)
    if method == "mrt":
        f = O.lbe_step(O.init_mrt_equilibrium(u), "mrt", nu, nsteps=steps)
    else:
        f = O.dugks_step(O.init_equilibrium(u), nu=nu, nsteps=steps)
    j = O.moments(f)[1]
    E_ref, st_ref = O.energy_spectrum(j, nu, n // 2)
    kr = resolved_shells(n, nu, st_ref["eps"])
    np.testing.assert_allclose(E[1:kr + 1], E_ref[1:kr + 1], rtol=1e-12)
    assert abs(st["K"] / st_ref["K"] - 1) < 1e-12 and abs(st["eps"] / st_ref["eps"] - 1) < 1e-12


def test_stability_ordering_of_the_schemes():
    """Sec. IV.E: on one mesh the DUGKS (CFL 0.9) stays stable at Reynolds
    numbers where the LBE blows up.  DHIT 32^3 (u' = 0.05, k0 = 4) over 1000
    time units: BGK-LBE blows up at nu = 1e-3 where MRT-LBE and the DUGKS
    run; MRT-LBE blows up at nu = 3e-6 where the DUGKS still runs."""
    from paper_1601_03815_amd import stability
    u = synth.dhit_field(32, seed=1, k0=4, u_rms=0.05)
    assert not stability.run_stable(u, "bgk", 1e-3, 1000.0)[0]
    assert stability.run_stable(u, "mrt", 1e-3, 1000.0)[0]
    assert stability.run_stable(u, "dugks", 1e-3, 1000.0)[0]
    assert not stability.run_stable(u, "mrt", 3e-6, 1000.0)[0]
    assert stability.run_stable(u, "dugks", 3e-6, 1000.0)[0]
    # Re_lambda of the initial field is proportional to 1/nu
    r1, r2 = stability.re_lambda(u, 1e-3), stability.re_lambda(u, 1e-4)
    assert abs(r2 / r1 - 10.0) < 1e-9
