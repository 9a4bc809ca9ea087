"""Sec. III statistics derived from the spectrum: closed forms on the CPU,
a recorded DHIT time series on the GPU."""
import math

import numpy as np
import pytest

from paper_1601_03815_amd.diagnostics import statistics


def test_single_mode_closed_forms():
    """u = U sin(kappa y) e_x, kappa = 2 pi m / n: K = U^2/4, eps = nu kappa^2 U^2/2,
    u' = U/sqrt(6), lambda = sqrt(5)/kappa, Re_lambda = u' lambda / nu,
    eta = (nu^3/eps)^(1/4), and D(k) is eps in shell m, zero elsewhere."""
    n, m, U, nu = 32, 3, 0.04, 0.01
    kappa = 2 * math.pi * m / n
    E = np.zeros(n // 2 + 1)
    E[m] = U * U / 4
    st = {"K": U * U / 4, "eps": nu * kappa ** 2 * U * U / 2, "S": 0.0, "F": 1.5}
    r = statistics(E, st, nu, n)
    assert r["u_rms"] == pytest.approx(U / math.sqrt(6), rel=1e-14)
    assert r["lambda"] == pytest.approx(math.sqrt(5) / kappa, rel=1e-14)
    assert r["re_lambda"] == pytest.approx(U / math.sqrt(6) * math.sqrt(5) / kappa / nu, rel=1e-14)
    assert r["eta"] == pytest.approx((nu ** 3 / st["eps"]) ** 0.25, rel=1e-14)
    assert r["kmax_eta"] == pytest.approx(math.pi * r["eta"], rel=1e-14)
    assert r["D"][m] == pytest.approx(st["eps"], rel=1e-14)
    assert np.count_nonzero(r["D"]) == 1


def test_dissipation_spectrum_sums_to_eps_for_on_shell_modes():
    """Modes whose |k| is an integer (axis modes) sit exactly on their shell,
    so sum_k D(k) equals eps = 2 nu sum |kappa|^2 E."""
    n, nu = 24, 0.003
    rng = np.random.default_rng(5)
    E = np.zeros(n // 2 + 1)
    E[1:9] = rng.uniform(0.0, 1e-3, 8)
    kappa = 2 * math.pi * np.arange(len(E)) / n
    eps = 2 * nu * np.sum(kappa ** 2 * E)
    r = statistics(E, {"K": E.sum(), "eps": eps, "S": 0.0, "F": 3.0}, nu, n)
    assert r["D"].sum() == pytest.approx(eps, rel=1e-13)


@pytest.mark.gpu
def test_recorded_dhit_statistics():
    """DHIT 32^3 (nu = 0.01, u' = 0.05, k0 = 4) over 300 MRT-LBE steps: the
    recorder samples every 50 steps; u' matches K; the dissipation spectrum
    sums to eps up to the shell rounding of off-axis modes; K decays, eta
    grows after the dissipation peak, and Re_lambda falls."""
    import paper_1601_03815_amd as dhit
    import synth
    from paper_1601_03815_amd.diagnostics import DhitStatistics
    nu = 0.01
    with dhit.Box(32, "mrt", "fp64", nu) as b:
        b.init_velocity_field(synth.dhit_field(32, seed=4, k0=4, u_rms=0.05))
        rec = DhitStatistics(b, nu).record(300, 50)
    assert [r["t"] for r in rec] == [0, 50, 100, 150, 200, 250, 300]
    for r in rec:
        assert r["u_rms"] == pytest.approx(math.sqrt(2 * r["K"] / 3), rel=1e-14)
        assert abs(r["D"].sum() / r["eps"] - 1) < 0.1
    K = [r["K"] for r in rec]
    assert all(a > b for a, b in zip(K, K[1:]))
    assert rec[-1]["re_lambda"] < rec[0]["re_lambda"]
    assert rec[-1]["eta"] > rec[2]["eta"]


class _FakeBox:
    """Stands in for a box: a fixed sequence of spectra, one per sample."""

    def __init__(self, stats, n=16):
        self.n, self._stats, self._i, self.steps = n, stats, 0, 0

    def energy_spectrum(self):
        st = self._stats[self._i]
        self._i += 1
        return np.array([0.0, st["K"]]), st

    def step(self, k):
        self.steps += k


def test_eddy_turnover_time():
    """t' = t eps0 / K0 with K0, eps0 of the first sample (Sec. IV.A)."""
    from paper_1601_03815_amd.diagnostics import DhitStatistics
    sts = [{"K": 2e-3, "eps": 4e-6, "S": 0.0, "F": 3.0}, {"K": 1.5e-3, "eps": 5e-6, "S": 0.0, "F": 3.0},
           {"K": 1e-3, "eps": 3e-6, "S": 0.0, "F": 3.0}]
    rec = DhitStatistics(_FakeBox(sts), 0.01).record(200, 100, dt=0.5)
    assert [r["t"] for r in rec] == [0.0, 50.0, 100.0]
    assert [r["t_prime"] for r in rec] == pytest.approx([0.0, 0.1, 0.2], rel=1e-14)


@pytest.mark.gpu
def test_normalized_slices_taylor_green():
    """Taylor-Green vortex on the plane z = L/2 (Z = pi): |u| / U =
    sqrt(sin^2 X cos^2 Y + cos^2 X sin^2 Y) and |omega| L / U =
    2 pi sqrt(cos^2 X sin^2 Y sin^2 Z + ... ) = 4 pi |sin X sin Y| there."""
    import paper_1601_03815_amd as dhit
    import synth
    from paper_1601_03815_amd.diagnostics import normalized_slices
    n, U = 16, 0.05
    x = synth.grid(n)
    Y, X = np.meshgrid(x, x, indexing="ij")
    with dhit.Box(n, "bgk", "fp64", 0.01) as b:
        b.init_velocity_field(synth.taylor_green(n, U))
        su, sw = normalized_slices(b, U)
    ref_u = np.sqrt(np.sin(X) ** 2 * np.cos(Y) ** 2 + np.cos(X) ** 2 * np.sin(Y) ** 2)
    assert np.abs(su - ref_u).max() < 1e-13
    assert np.abs(sw - 4 * np.pi * np.abs(np.sin(X) * np.sin(Y))).max() < 1e-11


def _table1():
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_parameters.json")))


def test_unit_conversion_reproduces_table1():
    """The paper's lattice runs are its spectral runs at velocity scale
    V_s = 0.0408 (Sec. IV.A, Table I): K0 and u'0 scale by V_s^2 and V_s
    (1.5383e-3 and 0.0320 as printed, to their 4-5 digits) and the viscosity
    by V_s n / (2 pi) (1.2395e-2 at 128^3 and 2.4790e-2 at 256^3 as printed;
    the conversion gives 1.2412e-2 and 2.4824e-2, 0.14% above: the printed
    pair corresponds to V_s = 0.04074, within the rounding of 0.0408)."""
    from paper_1601_03815_amd.diagnostics import lattice_viscosity
    t = _table1()
    vs, ps = t["v_s"], t["ps"]
    for n in ("128", "256"):
        lat = t["lattice"][n]
        assert vs ** 2 * ps["K0"] == pytest.approx(lat["K0"], rel=2e-4)
        assert vs * ps["u0"] == pytest.approx(lat["u0"], rel=1e-3)
        assert lattice_viscosity(ps["nu"], vs, int(n)) == pytest.approx(lat["nu"], rel=2e-3)
    assert t["lattice"]["256"]["nu"] == pytest.approx(2 * t["lattice"]["128"]["nu"], rel=1e-12)


def test_to_spectral_units_is_consistent():
    """The converted record satisfies the Sec. III relations in the new
    units: u' = sqrt(2K/3), lambda = sqrt(15 nu / eps) u', Re_lambda =
    u' lambda / nu, eta = (nu^3/eps)^(1/4), sum D = eps for on-shell
    modes; the dimensionless quantities are unchanged."""
    from paper_1601_03815_amd.diagnostics import statistics, to_spectral_units
    n, nu, vs = 64, 0.004, 0.0408
    E = np.zeros(n // 2 + 1)
    E[1:9] = np.random.default_rng(3).uniform(0.0, 1e-4, 8)
    kappa = 2 * math.pi * np.arange(len(E)) / n
    st = {"K": E.sum(), "eps": 2 * nu * np.sum(kappa ** 2 * E), "S": -0.4, "F": 4.0}
    rec = statistics(E, st, nu, n)
    rec.update(t=250.0, E=E, nu=nu, t_prime=1.7)
    sp = to_spectral_units(rec, vs, n)
    assert sp["u_rms"] == pytest.approx(math.sqrt(2 * sp["K"] / 3), rel=1e-13)
    assert sp["lambda"] == pytest.approx(math.sqrt(15 * sp["nu"] / sp["eps"]) * sp["u_rms"], rel=1e-13)
    assert sp["u_rms"] * sp["lambda"] / sp["nu"] == pytest.approx(rec["re_lambda"], rel=1e-13)
    assert sp["eta"] == pytest.approx((sp["nu"] ** 3 / sp["eps"]) ** 0.25, rel=1e-13)
    assert sp["D"].sum() == pytest.approx(sp["eps"], rel=1e-13)
    assert sp["E"].sum() == pytest.approx(sp["K"], rel=1e-13)
    ks = np.arange(len(E))  # spectral wavenumbers are the integer shells
    assert 2 * sp["nu"] * np.sum(ks ** 2 * sp["E"]) == pytest.approx(sp["eps"], rel=1e-13)
    for key in ("re_lambda", "kmax_eta", "S", "F", "t_prime"):
        assert sp[key] == rec[key]
    # time in units of the large-eddy time L/u is the same in both systems
    assert sp["t"] * sp["u_rms"] / (2 * math.pi) == pytest.approx(rec["t"] * rec["u_rms"] / n, rel=1e-13)
