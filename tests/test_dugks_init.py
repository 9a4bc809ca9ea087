"""Consistent initial state of the DUGKS (Sec. IV.A: the kinetic schemes start
from the non-equilibrium part that belongs to the initial velocity): the
oracle's first-order Chapman-Enskog start (`oracle.dugks_consistent_init`),
pinned on the CPU to closed forms and to the scheme's own dynamics, and the
library's `init_consistent` for DUGKS boxes against it on the GPU.
"""
import numpy as np
import pytest

import oracle as O
import synth

RT = 1.0 / 3.0


def _shear_wave(n, U):
    u = np.zeros((3, n, n, n))
    y = np.arange(n)
    u[0] = U * np.sin(2 * np.pi * y / n)[None, :, None]
    return u


def _stress_neq(f, rho0=1.0):
    """Pi_ab of f - f^eq(drho, j) for every cell: [3, 3, n, n, n]."""
    c, _ = O.lattice()
    d, j, _ = O.moments(f, rho0)
    g = f - O.init_equilibrium(j / rho0, d, rho0)
    return np.einsum("ia,ib,i...->ab...", c, c, g)


def test_velocity_gradient_taylor_green_closed_form():
    """Spectral d_a u_b of the Taylor-Green vortex against its closed form
    (x_i = 2 pi i / n, so d/dx per cell carries kappa = 2 pi / n)."""
    n, U = 16, 0.05
    u = synth.taylor_green(n, U)
    G = O.velocity_gradient(u)
    x = 2 * np.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    k = 2 * np.pi / n
    ref = np.zeros_like(G)
    ref[0, 0] = U * k * np.cos(X) * np.cos(Y) * np.cos(Z)
    ref[1, 0] = -U * k * np.sin(X) * np.sin(Y) * np.cos(Z)
    ref[2, 0] = -U * k * np.sin(X) * np.cos(Y) * np.sin(Z)
    ref[0, 1] = U * k * np.sin(X) * np.sin(Y) * np.cos(Z)
    ref[1, 1] = -U * k * np.cos(X) * np.cos(Y) * np.cos(Z)
    ref[2, 1] = U * k * np.cos(X) * np.sin(Y) * np.sin(Z)
    assert np.abs(G - ref).max() <= 1e-15


def test_uniform_flow_starts_at_equilibrium():
    n = 6
    u = np.zeros((3, n, n, n))
    u[0], u[1], u[2] = 0.02, -0.01, 0.03
    f = O.dugks_consistent_init(u, nu=0.01)
    np.testing.assert_allclose(f, O.init_equilibrium(u), rtol=0, atol=1e-18)


@pytest.mark.parametrize("nu,dt", [(0.01, 0.5), (0.05, 0.35)])
def test_moments_and_viscous_stress(nu, dt):
    """The start keeps drho and j of the equilibrium (the Chapman-Enskog
    part carries no mass or momentum) and its non-equilibrium stress is the
    viscous stress scaled by the f -> f~ map: -(tau + dt/2) rho0 RT
    (d_a u_b + d_b u_a), tau = nu/RT (lattice isotropy to fourth order
    turns W (xi xi - RT I) into that); for the shear wave u_x = U sin(k y)
    the only component is the closed form -(tau + dt/2) rho0 RT U k cos(k y)."""
    n, U, rho0 = 16, 1e-3, 1.0
    tau = nu / RT
    u = _shear_wave(n, U)
    drho = 1e-4 * np.cos(2 * np.pi * np.arange(n) / n)[:, None, None] * np.ones((n, n, n))
    f = O.dugks_consistent_init(u, drho, nu=nu, dt=dt, rho0=rho0)
    d, j, _ = O.moments(f, rho0)
    assert np.abs(d - drho).max() <= 1e-18
    assert np.abs(j - rho0 * u).max() <= 1e-18
    P = _stress_neq(f, rho0)
    k = 2 * np.pi / n
    ref = np.zeros_like(P)
    ref[0, 1] = ref[1, 0] = -(tau + dt / 2) * rho0 * RT * U * k * np.cos(k * np.arange(n))[None, :, None]
    assert np.abs(P - ref).max() <= 1e-13 * np.abs(ref).max()
    # a general field: the same identity with the spectral gradient
    v = synth.dhit_field(8, seed=4, k0=2, u_rms=0.05)
    g = O.dugks_consistent_init(v, nu=nu, dt=dt)
    G = O.velocity_gradient(v)
    Pg = _stress_neq(g)
    refg = -(tau + dt / 2) * RT * (G + G.transpose(1, 0, 2, 3, 4))
    assert np.abs(Pg - refg).max() <= 1e-12 * np.abs(refg).max()


@pytest.mark.parametrize("nu", [0.05, 0.01, 0.002])
def test_start_is_the_schemes_slaved_state(nu):
    """A shear wave started from the Chapman-Enskog state keeps its
    non-equilibrium stress at the value its own velocity implies, step after
    step (within the scheme's O((k dx)^2) error: 2%): the state is the one
    the DUGKS relaxes to.  Started from equilibrium instead, the stress is
    zero at t = 0 and overshoots by more than 20% after one step; for
    tau < h/2, where the transform coefficient (2 tau - h)/(2 tau + dt) is
    negative, it then flips about the slaved value every step, off by more
    than 20% in each of the first three steps.  A missing factor
    1 + dt/(2 tau) or a wrong sign also fails the first bound."""
    n, U, dt = 32, 1e-4, 0.5
    tau = nu / RT
    k = 2 * np.pi / n
    y = np.arange(n)
    u = _shear_wave(n, U)

    def ratios(f, steps=4):
        out = []
        for _ in range(steps):
            _, j, _ = O.moments(f)
            amp = 2 * np.mean(j[0] * np.sin(k * y)[None, :, None])
            slaved = -(tau + dt / 2) * RT * amp * k
            pxy = _stress_neq(f)[0, 1]
            out.append(2 * np.mean(pxy * np.cos(k * y)[None, :, None]) / slaved)
            f = O.dugks_step(f, nu=nu, dt=dt)
        return np.array(out)

    ce = ratios(O.dugks_consistent_init(u, nu=nu, dt=dt))
    eq = ratios(O.init_equilibrium(u))
    assert np.all(np.abs(ce - 1) <= 0.02), ce
    assert abs(eq[0]) <= 1e-12 and abs(eq[1] - 1) > 0.2, eq
    if tau < dt / 4:
        assert np.all(np.abs(eq[1:] - 1) > 0.2), eq
