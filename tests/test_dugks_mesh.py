"""DUGKS on a stretched periodic mesh (the paper's reason for the finite-
volume scheme, Sec. V; the reconstruction of Sec. II.A written with the cell
and face positions of a non-uniform mesh).  CPU: the oracle pinned to the
uniform scheme, a scaling identity, conservation, exact free transport of
bilinear data and second-order convergence of a shear wave's decay; GPU:
the library's mesh path against the oracle."""
import numpy as np
import pytest

import synth

AMP = (0.2, 0.3, 0.25)


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_oracle_unit_widths_is_the_uniform_scheme():
    import oracle as O
    n = 6
    f0 = synth.random_populations(n, seed=11, amplitude=0.01)
    a = O.dugks_step_mesh(f0, np.ones((3, n)), nu=0.02, dt=0.5, nsteps=2)
    b = O.dugks_step(f0, nu=0.02, dt=0.5, nsteps=2)
    assert _rel(a, b) < 1e-14


def test_oracle_uniform_spacing_scaling():
    """A uniform mesh of spacing c with (tau, dt) is the unit mesh with
    (tau/c, dt/c): lengths only enter through dt/dx and tau/dx."""
    import oracle as O
    n, c = 6, 0.75
    f0 = synth.random_populations(n, seed=12, amplitude=0.01)
    a = O.dugks_step_mesh(f0, np.full((3, n), c), tau=0.06, dt=0.3)
    b = O.dugks_step(f0, tau=0.06 / c, dt=0.3 / c)
    assert _rel(a, b) < 1e-14


def test_oracle_mesh_conservation_and_uniform_flow():
    """Mass and momentum weighted by the cell volumes are conserved (the
    face fluxes telescope); a uniform flow stays exactly uniform."""
    import oracle as O
    n = 7
    W = synth.stretched_widths(n, AMP)
    V = W[0][None, None, :] * W[1][None, :, None] * W[2][:, None, None]
    f0 = synth.random_populations(n, seed=13, amplitude=0.01)
    f1 = O.dugks_step_mesh(f0, W, nu=0.05, dt=0.3, nsteps=3)
    d0, j0, _ = O.moments(f0)
    d1, j1, _ = O.moments(f1)
    scale = np.abs(f0).sum()
    assert abs((V * d1).sum() - (V * d0).sum()) < 1e-14 * scale
    assert np.abs((V * j1).sum(axis=(1, 2, 3)) - (V * j0).sum(axis=(1, 2, 3))).max() < 1e-14 * scale
    g0 = O.init_equilibrium(synth.uniform_flow(n, 0.03, -0.02, 0.01))
    g1 = O.dugks_step_mesh(g0, W, nu=0.05, dt=0.3, nsteps=3)
    assert np.abs(g1 - g0).max() < 1e-17


def test_oracle_mesh_free_transport_of_bilinear_data_is_exact():
    """Collisionless limit (tau -> inf): the linear reconstruction at the
    face position x_b = c_L + w_L/2 with the gradient (f_R - f_L)/(c_R - c_L),
    the tangential gradients interpolated with the same weight, and the half
    step h xi . sigma reproduce free transport f(x - xi dt) exactly for data
    of the form a + b.x + (xy, yz, xz terms); checked on the cells whose
    stencil does not cross the periodic wrap.  (Placing the face midway
    between the centres, or taking the plain mean of the tangential
    gradients, breaks this by 1e-4 and 2e-6 on this mesh.)"""
    import oracle as O
    n, dt = 10, 0.3
    W = synth.stretched_widths(n, AMP)
    c = [synth.cell_centres(W[a]) for a in range(3)]
    Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    xi, _w = O.lattice()
    coef = np.random.default_rng(1).uniform(-1e-3, 1e-3, (19, 7))

    def poly(q, X, Y, Z):
        a = coef[q]
        return a[0] + a[1] * X + a[2] * Y + a[3] * Z + a[4] * X * Y + a[5] * Y * Z + a[6] * X * Z

    f0 = np.stack([poly(q, X, Y, Z) for q in range(19)])
    f1 = O.dugks_step_mesh(f0, W, tau=1e13, dt=dt)
    ref = np.stack([poly(q, X - xi[q, 0] * dt, Y - xi[q, 1] * dt, Z - xi[q, 2] * dt) for q in range(19)])
    inner = (slice(None), slice(1, n - 1), slice(1, n - 1), slice(1, n - 1))
    assert np.abs(f1[inner] - ref[inner]).max() < 1e-12 * np.abs(ref).max()


def test_oracle_mesh_shear_wave_second_order():
    """u_x = U sin(2 pi y/L) at the cell centres of a stretched mesh
    (widths varying by 1.5-1.9x on each axis), CFL 0.9 on the smallest cell:
    the decay rate after the start-up layer converges to nu kappa^2 at
    second order (8^3 -> 16^3)."""
    import oracle as O
    nu, U = 0.1, 1e-3
    errs = []
    for n in (8, 16):
        W = synth.stretched_widths(n, AMP)
        dt = 0.9 * W.min() / np.sqrt(2.0)
        L = float(n)
        kap = 2 * np.pi / L
        T = 0.4 / (nu * kap * kap)
        s1 = int(round(T / 4 / dt))
        s2 = int(round(T / dt)) - s1
        sn = np.sin(2 * np.pi * synth.cell_centres(W[1]) / L)

        def amp(f):
            return 2.0 / L * np.sum(W[1] * O.moments(f)[1][0].mean(axis=(0, 2)) * sn)

        g1 = O.dugks_step_mesh(O.init_equilibrium(synth.shear_wave_on_mesh(W, U)), W, nu=nu, dt=dt, nsteps=s1)
        g = O.dugks_step_mesh(g1, W, nu=nu, dt=dt, nsteps=s2)
        errs.append(abs(-np.log(amp(g) / amp(g1)) / (s2 * dt) / (nu * kap * kap) - 1))
    assert errs[1] < 0.05, errs
    assert 3.3 < errs[0] / errs[1] < 6.0, errs


def _volumes(W):
    return W[0][None, None, :] * W[1][None, :, None] * W[2][:, None, None]


def _weighted_sums(f, W):
    import oracle as O
    d, j, _ = O.moments(f)
    V = _volumes(W)
    return np.array([(V * d).sum(), (V * j[0]).sum(), (V * j[1]).sum(), (V * j[2]).sum(),
                     0.5 * (V * np.sum(j * j, axis=0)).sum()])


@pytest.mark.gpu
@pytest.mark.parametrize("n", [4, 5, 12, 17, 32])
def test_mesh_step_parity_fp64(n):
    """Two steps from a random state on a stretched mesh, element by
    element within 1e-12 of the oracle, with the volume-weighted sums of the
    step history and of moments()."""
    import oracle as O
    import paper_1601_03815_amd as dhit
    W = synth.stretched_widths(n, AMP)
    nu, dt = 0.02, 0.6 * W.min() / np.sqrt(2.0)
    f0 = synth.random_populations(n, seed=300 + n, amplitude=0.01)
    with dhit.Box(n, "dugks", "fp64", nu, dt=dt) as b:
        b.set_mesh(W)
        b.set_populations(f0)
        b.step(2)
        got = b.get_populations()
        hist = b.sums_history(2)
        _d, _j, sums = b.moments(want_fields=False)
    f1 = O.dugks_step_mesh(f0, W, nu=nu, dt=dt)
    ref = O.dugks_step_mesh(f1, W, nu=nu, dt=dt)
    assert _rel(got, ref) <= 1e-12
    scale = np.abs(f0).sum() * W.max() ** 3
    assert np.abs(hist[0] - _weighted_sums(f1, W)).max() <= 1e-12 * scale
    assert np.abs(hist[1] - _weighted_sums(ref, W)).max() <= 1e-12 * scale
    assert np.abs(sums - _weighted_sums(ref, W)).max() <= 1e-12 * scale


@pytest.mark.gpu
@pytest.mark.parametrize("n", [5, 16])
def test_mesh_step_parity_fp32(n):
    import oracle as O
    import paper_1601_03815_amd as dhit
    W = synth.stretched_widths(n, AMP)
    nu, dt = 0.02, 0.6 * W.min() / np.sqrt(2.0)
    f0 = synth.random_populations(n, seed=400 + n, amplitude=0.01).astype(np.float32).astype(np.float64)
    with dhit.Box(n, "dugks", "fp32", nu, dt=dt) as b:
        b.set_mesh(W)
        b.set_populations(f0)
        b.step(1)
        got = b.get_populations()
    assert _rel(got, O.dugks_step_mesh(f0, W, nu=nu, dt=dt)) <= 2e-6


@pytest.mark.gpu
def test_mesh_shear_wave_second_order_on_the_gpu():
    """The shear-wave decay rate on the stretched mesh at 16^3 and 32^3
    (sizes the oracle takes a minute for): second-order convergence, the
    oracle's 16^3 error reproduced."""
    import oracle as O
    import paper_1601_03815_amd as dhit
    nu, U = 0.1, 1e-3
    errs = []
    for n in (16, 32):
        W = synth.stretched_widths(n, AMP)
        dt = 0.9 * W.min() / np.sqrt(2.0)
        L = float(n)
        kap = 2 * np.pi / L
        T = 0.4 / (nu * kap * kap)
        s1 = int(round(T / 4 / dt))
        s2 = int(round(T / dt)) - s1
        sn = np.sin(2 * np.pi * synth.cell_centres(W[1]) / L)
        with dhit.Box(n, "dugks", "fp64", nu, dt=dt) as b:
            b.set_mesh(W)
            b.init_velocity_field(synth.shear_wave_on_mesh(W, U))
            b.step(s1)
            a1 = 2.0 / L * np.sum(W[1] * b.moments()[1][0].mean(axis=(0, 2)) * sn)
            b.step(s2)
            a2 = 2.0 / L * np.sum(W[1] * b.moments()[1][0].mean(axis=(0, 2)) * sn)
        errs.append(abs(-np.log(a2 / a1) / (s2 * dt) / (nu * kap * kap) - 1))
    assert abs(errs[0] - 0.03419) < 1e-4, errs
    assert 3.3 < errs[0] / errs[1] < 6.0, errs


@pytest.mark.gpu
def test_mesh_validation_and_reset():
    """Errors: an LBE box, a width <= 0 or not finite, CFL above 1; a mesh
    box in a batch and in the spectral diagnostics.  set_mesh(None) returns
    the box to the uniform scheme (same state as a box that never had a
    mesh), and unit widths give the uniform scheme."""
    import oracle as O
    import paper_1601_03815_amd as dhit
    n = 8
    W = synth.stretched_widths(n, AMP)
    dt = 0.6 * W.min() / np.sqrt(2.0)
    with dhit.Box(n, "mrt", "fp64", 0.01) as lbe:
        with pytest.raises(dhit.DhitError) as e:
            lbe.set_mesh(W)
        assert e.value.code == -4
    f0 = synth.random_populations(n, seed=500, amplitude=0.01)
    with dhit.Box(n, "dugks", "fp64", 0.02, dt=dt) as b, dhit.Box(n, "dugks", "fp64", 0.02, dt=dt) as c:
        for bad in (np.where(np.arange(3 * n).reshape(3, n) == 5, 0.0, W), np.where(W > 1.2, np.nan, W),
                    W * (dt * np.sqrt(2.0) / W.min()) * 0.99):
            with pytest.raises(dhit.DhitError) as e:
                b.set_mesh(bad)
            assert e.value.code == -1
        b.set_mesh(W)
        with pytest.raises(dhit.DhitError) as e:
            b.energy_spectrum()
        assert e.value.code == -4
        with pytest.raises(dhit.DhitError) as e:
            b.vorticity()
        assert e.value.code == -4
        with pytest.raises(dhit.DhitError):
            dhit.step_batch([b.handle, c.handle], 1)
        b.set_mesh(None)
        bt = dhit.create_batch([b.handle, c.handle], autotune=False)
        try:
            b.set_mesh(W)   # after the batch was built
            with pytest.raises(dhit.DhitError) as e:
                dhit.batch_step(bt, 1)
            assert e.value.code == -1
        finally:
            dhit.destroy_batch(bt)
        b.set_mesh(W)
        b.set_mesh(np.ones((3, n)))
        b.set_populations(f0)
        b.step(1)
        assert _rel(b.get_populations(), O.dugks_step(f0, nu=0.02, dt=dt)) <= 1e-12
        b.set_mesh(None)
        b.set_populations(f0)
        c.set_populations(f0)
        b.step(1)
        c.step(1)
        assert np.array_equal(b.get_populations(), c.get_populations())


@pytest.mark.gpu
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_mesh_conservation_256(precision, tol):
    """256^3 DHIT field on the stretched mesh (the benchmark's grid), 20
    steps at CFL 0.9: the volume-weighted mass and momentum of the step
    history stay at their initial values (the oracle's conservation pin, at
    a size it cannot run); the weighted kinetic energy decays."""
    import paper_1601_03815_amd as dhit
    n = 256
    W = synth.stretched_widths(n, AMP)
    dt = 0.9 * W.min() / np.sqrt(2.0)
    with dhit.Box(n, "dugks", precision, 0.01, dt=dt) as b:
        b.set_mesh(W)
        b.init_velocity_field(synth.dhit_field(n, seed=1, k0=4, u_rms=0.05))
        _d, _j, s0 = b.moments(want_fields=False)
        b.step(20)
        h = b.sums_history(20)
    scale = 0.05 * float(n) ** 3  # |u| ~ u' summed over the volume
    assert np.abs(h[:, 0:4] - s0[0:4]).max() <= tol * scale, np.abs(h[:, 0:4] - s0[0:4]).max()
    assert np.all(np.diff(h[:, 4]) < 0)


@pytest.mark.gpu
def test_mesh_fp32_energy_tracks_fp64():
    """FP32 (deviation form, compensated moment sums) on the stretched mesh:
    over 400 steps of a 64^3 DHIT field (K decays to 39%), the volume-weighted
    kinetic energy of every step stays within 5e-6 of the FP64 run's
    (measured 5.5e-7)."""
    import paper_1601_03815_amd as dhit
    n, steps = 64, 400
    W = synth.stretched_widths(n, AMP)
    dt = 0.9 * W.min() / np.sqrt(2.0)
    u = synth.dhit_field(n, seed=1, k0=4, u_rms=0.05)
    K = {}
    for prec in ("fp64", "fp32"):
        with dhit.Box(n, "dugks", prec, 0.01, dt=dt) as b:
            b.set_mesh(W)
            b.init_velocity_field(u)
            b.step(steps)
            K[prec] = b.sums_history(steps)[:, 4]
    assert K["fp64"][-1] < 0.5 * K["fp64"][0]
    assert np.max(np.abs(K["fp32"] - K["fp64"]) / K["fp64"]) < 5e-6
