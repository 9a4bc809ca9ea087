"""Vorticity of the velocity field (the flow fields of Sec. IV.B): the
oracle's spectral curl against closed forms on the CPU; the library's
against the oracle on the GPU."""
import numpy as np
import pytest

import synth


def test_oracle_vorticity_taylor_green_closed_form():
    """Taylor-Green vortex in lattice units (X = 2 pi x/n, d/dx = (2 pi/n) d/dX):
    omega = (2 pi/n) U (-cos X sin Y sin Z, -sin X cos Y sin Z, 2 sin X sin Y cos Z)."""
    import oracle
    n, U = 16, 0.05
    x = synth.grid(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    a = 2 * np.pi / n * U
    ref = np.stack([-a * np.cos(X) * np.sin(Y) * np.sin(Z), -a * np.sin(X) * np.cos(Y) * np.sin(Z),
                    2 * a * np.sin(X) * np.sin(Y) * np.cos(Z)])
    w = oracle.vorticity(synth.taylor_green(n, U))
    assert np.abs(w - ref).max() < 1e-15


@pytest.mark.parametrize("n", [15, 16])
def test_oracle_vorticity_enstrophy_and_divergence(n):
    """Solenoidal periodic field: <|omega|^2> = eps / nu (eps of the
    spectrum, Sec. III) and div omega = 0; a uniform flow has none."""
    import oracle
    nu = 0.01
    u = synth.dhit_field(n, seed=7, k0=2, u_rms=0.05)
    w = oracle.vorticity(u)
    _E, st = oracle.energy_spectrum(u, nu)
    assert abs(np.mean(np.sum(w * w, axis=0)) - st["eps"] / nu) < 1e-12 * st["eps"] / nu
    wh = np.fft.fftn(w, axes=(1, 2, 3))
    k1 = np.fft.fftfreq(n, 1.0 / n)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    div = kx * wh[0] + ky * wh[1] + kz * wh[2]
    assert np.abs(div).max() < 1e-12 * np.abs(wh).max()
    assert np.abs(oracle.vorticity(synth.uniform_flow(n, 0.03, -0.02, 0.01))).max() < 1e-17


@pytest.mark.gpu
@pytest.mark.parametrize("method,precision", [("mrt", "fp64"), ("dugks", "fp64"), ("bgk", "fp32")])
@pytest.mark.parametrize("n", [15, 16, 32])
def test_vorticity_parity(method, precision, n):
    """The library's curl of a box's velocity after a few steps against the
    oracle's curl of the same velocity (the box's moments), element by
    element: odd n (no Nyquist plane) and even n (Nyquist derivatives
    dropped), within 1e-12 of the largest |omega|."""
    import oracle
    import paper_1601_03815_amd as dhit
    with dhit.Box(n, method, precision, 0.01) as b:
        b.init_velocity_field(synth.dhit_field(n, seed=8, k0=2, u_rms=0.05))
        b.step(3)
        got = b.vorticity()
        _d, j, _s = b.moments()
    ref = oracle.vorticity(j)  # u = j / rho0 with rho0 = 1
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.gpu
def test_vorticity_parity_128():
    """128^3 MRT box after 3 steps: every element within 1e-12 of the oracle."""
    import oracle
    import paper_1601_03815_amd as dhit
    n = 128
    with dhit.Box(n, "mrt", "fp64", 0.005) as b:
        b.init_velocity_field(synth.dhit_field(n, seed=1, k0=4, u_rms=0.05))
        b.step(3)
        got = b.vorticity()
        _d, j, _s = b.moments()
    ref = oracle.vorticity(j)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.gpu
@pytest.mark.parametrize("method", ["mrt", "dugks"])
def test_vorticity_enstrophy_256(method):
    """256^3, the benchmark's field and viscosity, after 4 steps: the
    library's curl and its spectrum (two separate code paths: inverse
    transforms of i kappa x u_hat against kappa^2-weighted shell sums) obey
    <|omega|^2> + <(div u)^2> = eps / nu (|kappa|^2 |u_hat|^2 = |kappa x u_hat|^2
    + |kappa . u_hat|^2 mode by mode; the flow is weakly compressible, so
    the divergence term, 2e-3 of eps/nu here, is needed), to 1e-10."""
    import paper_1601_03815_amd as dhit
    n, nu = 256, 0.0025
    with dhit.Box(n, method, "fp64", nu) as b:
        b.init_velocity_field(synth.dhit_field(n, seed=1, k0=4, u_rms=0.05))
        b.step(4)
        w = b.vorticity()
        _E, st = b.energy_spectrum()
        _d, j, _s = b.moments()
    ens = float(np.mean(np.sum(w * w, axis=0)))
    del w
    k1 = np.fft.fftfreq(n, 1.0 / n)
    k1 = np.where(np.abs(k1) == n // 2, 0.0, k1) * (2 * np.pi / n)
    div_h = np.zeros((n, n, n), dtype=np.complex128)
    for a in range(3):
        shape = [1, 1, 1]
        shape[2 - a] = n   # axis 2 is x, 1 is y, 0 is z
        div_h += 1j * k1.reshape(shape) * np.fft.fftn(j[a])
    div2 = float(np.mean(np.fft.ifftn(div_h).real ** 2))
    ref = st["eps"] / nu
    assert abs(ens + div2 - ref) <= 1e-10 * ref, (ens, div2, ref)
    assert div2 < 0.01 * ref


@pytest.mark.gpu
@pytest.mark.parametrize("n", [4, 9])
def test_vorticity_of_uniform_flow_is_zero(n):
    """Degenerate case: a uniform flow (only the k = 0 mode) has no
    vorticity; smallest grids, odd and even."""
    import paper_1601_03815_amd as dhit
    with dhit.Box(n, "bgk", "fp64", 0.01) as b:
        b.init_velocity_field(synth.uniform_flow(n, 0.03, -0.02, 0.01))
        w = b.vorticity()
    assert w.shape == (3, n, n, n)
    assert np.abs(w).max() < 1e-17
