"""Plain FP64 CPU oracle for the LBE and DUGKS steps of arXiv 1601.03815.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports, links
or calls anything here, and nothing here comes from the GPU library.

Arrays follow one convention: a population field is a C-contiguous float64
array of shape (19, n, n, n) indexed [q, z, y, x]; a velocity field is
(3, n, n, n).  Lattice units throughout (dx = 1, c = 1, RT = 1/3).

The time-stepping kernels are plain C loops (``dhit_oracle.c``); the spectral
diagnostics of Sec. III are written here with numpy's FFT as the library
primitive.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

Q = 19


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        d = ctypes.c_double
        i32 = ctypes.c_int32
        i64 = ctypes.c_int64
        p = ctypes.c_void_p
        sig = {
            "oracle_version": ([], ctypes.c_int),
            "oracle_lattice": ([p, p], None),
            "oracle_feq": ([d, d, d, d, d, p], None),
            "oracle_mrt_matrix": ([p], None),
            "oracle_mrt_inverse": ([p, p], None),
            "oracle_mrt_meq": ([d, d, d, d, d, d, d, d, p], None),
            "oracle_collide_bgk": ([p, i32, d, d], None),
            "oracle_collide_mrt": ([p, i32, p, d, d, d, d], None),
            "oracle_stream": ([p, p, i32], None),
            "oracle_lbe_step": ([p, p, i32, i32, d, p, d, d, d, d], None),
            "oracle_dugks_transform": ([p, p, p, i32, d, d, d], None),
            "oracle_dugks_step": ([p, p, i32, d, d, d], None),
            "oracle_dugks_cells": ([p, i32, d, d, d, p, i64, p], None),
            "oracle_dugks_step_mesh": ([p, p, i32, p, d, d, d], None),
            "oracle_lbe_pull_cells": ([p, i32, i32, d, p, d, d, d, d, p, i64, p], None),
            "oracle_moments": ([p, i32, d, p, p, p], None),
            "oracle_init_equilibrium": ([p, i32, p, p, d], None),
            "oracle_init_mrt_equilibrium": ([p, i32, p, p, d, d, d, d], None),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _LIB = lib
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (shape, a.shape))
    return a


def _n_of(f):
    if f.ndim != 4 or f.shape[0] != Q or not (f.shape[1] == f.shape[2] == f.shape[3]):
        raise ValueError("population field must have shape (19, n, n, n), got %s" % (f.shape,))
    return f.shape[1]


# ----------------------------------------------------------------------------
# Parameters (Sec. II.B and Sec. IV.A)
# ----------------------------------------------------------------------------

#: MRT constants used in the paper (Sec. IV.A).
PAPER_MRT = dict(s1=1.19, s2=1.4, s4=1.2, s10=1.4, s16=1.98,
                 w_eps=0.0, w_epsj=-475.0 / 63.0, w_xx=0.0)


def tau_lbe(nu):
    """BGK-LBE relaxation time: nu = (1/3)(tau - 1/2) with dt = dx = 1
    (the viscosity relation of Sec. II.B with s9 = 1/tau)."""
    return 3.0 * nu + 0.5


def tau_dugks(nu):
    """DUGKS relaxation time of the continuous BGK model, nu = tau RT."""
    return 3.0 * nu


def mrt_rates(nu, s1=1.19, s2=1.4, s4=1.2, s10=1.4, s16=1.98, s9=None, s13=None, dt=1.0):
    """Diagonal of S in the order of Sec. II.B; s9 = s13 = dt/(3 nu + dt/2)
    unless given."""
    if s9 is None:
        s9 = dt / (3.0 * nu + 0.5 * dt)
    if s13 is None:
        s13 = s9
    return np.array([0.0, s1, s2, 0.0, s4, 0.0, s4, 0.0, s4,
                     s9, s10, s9, s10, s13, s13, s13, s16, s16, s16])


# ----------------------------------------------------------------------------
# Lattice, equilibrium, MRT transformation
# ----------------------------------------------------------------------------

def lattice():
    c = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q)
    _lib().oracle_lattice(_ptr(c), _ptr(w))
    return c, w


def feq(drho, jx, jy, jz, rho0=1.0):
    out = np.zeros(Q)
    _lib().oracle_feq(drho, jx, jy, jz, rho0, _ptr(out))
    return out


def mrt_matrix():
    M = np.zeros((Q, Q))
    _lib().oracle_mrt_matrix(_ptr(M))
    return M


def mrt_inverse(M):
    M = _f64(M, (Q, Q))
    Mi = np.zeros((Q, Q))
    _lib().oracle_mrt_inverse(_ptr(M), _ptr(Mi))
    return Mi


def mrt_meq(drho, jx, jy, jz, rho0=1.0, w_eps=0.0, w_epsj=-475.0 / 63.0, w_xx=0.0):
    out = np.zeros(Q)
    _lib().oracle_mrt_meq(drho, jx, jy, jz, rho0, w_eps, w_epsj, w_xx, _ptr(out))
    return out


# ----------------------------------------------------------------------------
# LBE
# ----------------------------------------------------------------------------

def collide_bgk(f, tau, rho0=1.0):
    f = _f64(f).copy()
    _lib().oracle_collide_bgk(_ptr(f), _n_of(f), tau, rho0)
    return f


def collide_mrt(f, s, w_eps=0.0, w_epsj=-475.0 / 63.0, w_xx=0.0, rho0=1.0):
    f = _f64(f).copy()
    s = _f64(s, (Q,))
    _lib().oracle_collide_mrt(_ptr(f), _n_of(f), _ptr(s), w_eps, w_epsj, w_xx, rho0)
    return f


def stream(f):
    f = _f64(f)
    g = np.empty_like(f)
    _lib().oracle_stream(_ptr(f), _ptr(g), _n_of(f))
    return g


def lbe_step(f, method, nu, rho0=1.0, mrt=None, nsteps=1):
    """`nsteps` LBE steps (collide then stream) from the pre-collision state.
    method: 'bgk' or 'mrt'.  `mrt` overrides entries of PAPER_MRT and may
    carry an explicit 's' array."""
    f = _f64(f)
    n = _n_of(f)
    m = dict(PAPER_MRT)
    if mrt:
        m.update(mrt)
    s = m.get("s")
    if s is None:
        s = mrt_rates(nu, m["s1"], m["s2"], m["s4"], m["s10"], m["s16"])
    s = _f64(s, (Q,))
    meth = {"bgk": 0, "mrt": 1}[method]
    cur = f.copy()
    out = np.empty_like(f)
    for _ in range(nsteps):
        _lib().oracle_lbe_step(_ptr(cur), _ptr(out), n, meth, tau_lbe(nu), _ptr(s),
                               m["w_eps"], m["w_epsj"], m["w_xx"], rho0)
        cur, out = out, cur
    return cur


def collide(f, method, nu, rho0=1.0, mrt=None):
    """The collision of `lbe_step` alone (used to compare with a solver that
    stores post-collision populations)."""
    m = dict(PAPER_MRT)
    if mrt:
        m.update(mrt)
    if method == "bgk":
        return collide_bgk(f, tau_lbe(nu), rho0)
    s = m.get("s")
    if s is None:
        s = mrt_rates(nu, m["s1"], m["s2"], m["s4"], m["s10"], m["s16"])
    return collide_mrt(f, s, m["w_eps"], m["w_epsj"], m["w_xx"], rho0)


def lbe_pull_cells(fpost, cells, method, nu, rho0=1.0, mrt=None):
    """Pull-form update of selected flat cell indices from a post-collision
    field: returns (len(cells), 19)."""
    fpost = _f64(fpost)
    n = _n_of(fpost)
    m = dict(PAPER_MRT)
    if mrt:
        m.update(mrt)
    s = m.get("s")
    if s is None:
        s = mrt_rates(nu, m["s1"], m["s2"], m["s4"], m["s10"], m["s16"])
    s = _f64(s, (Q,))
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((len(cells), Q))
    _lib().oracle_lbe_pull_cells(_ptr(fpost), n, {"bgk": 0, "mrt": 1}[method], tau_lbe(nu),
                                 _ptr(s), m["w_eps"], m["w_epsj"], m["w_xx"], rho0,
                                 _ptr(cells), len(cells), _ptr(out))
    return out


# ----------------------------------------------------------------------------
# DUGKS
# ----------------------------------------------------------------------------

def dugks_transform(ft, tau, dt=0.5, rho0=1.0):
    ft = _f64(ft)
    fbp = np.empty_like(ft)
    ftp = np.empty_like(ft)
    _lib().oracle_dugks_transform(_ptr(ft), _ptr(fbp), _ptr(ftp), _n_of(ft), tau, dt, rho0)
    return fbp, ftp


def dugks_step(ft, nu=None, dt=0.5, rho0=1.0, nsteps=1, tau=None):
    ft = _f64(ft)
    if tau is None:
        tau = tau_dugks(nu)
    cur = ft.copy()
    out = np.empty_like(ft)
    for _ in range(nsteps):
        _lib().oracle_dugks_step(_ptr(cur), _ptr(out), _n_of(ft), tau, dt, rho0)
        cur, out = out, cur
    return cur


def dugks_step_mesh(ft, widths, nu=None, dt=0.5, rho0=1.0, nsteps=1, tau=None):
    """`nsteps` DUGKS steps on a stretched periodic mesh: widths[a][i] is
    the width of cell i along axis a (x, y, z).  With unit widths this is
    `dugks_step`."""
    ft = _f64(ft)
    n = _n_of(ft)
    W = _f64(widths, (3, n))
    if tau is None:
        tau = tau_dugks(nu)
    cur = ft.copy()
    out = np.empty_like(ft)
    for _ in range(nsteps):
        _lib().oracle_dugks_step_mesh(_ptr(cur), _ptr(out), n, _ptr(W), tau, dt, rho0)
        cur, out = out, cur
    return cur


def dugks_cells(ft, cells, nu=None, dt=0.5, rho0=1.0, tau=None):
    ft = _f64(ft)
    if tau is None:
        tau = tau_dugks(nu)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((len(cells), Q))
    _lib().oracle_dugks_cells(_ptr(ft), _n_of(ft), tau, dt, rho0, _ptr(cells), len(cells), _ptr(out))
    return out


# ----------------------------------------------------------------------------
# Moments and initial states
# ----------------------------------------------------------------------------

def moments(f, rho0=1.0):
    """(drho[n,n,n], j[3,n,n,n], sums[5]) with sums = (sum drho, sum jx,
    sum jy, sum jz, 1/2 sum |u|^2)."""
    f = _f64(f)
    n = _n_of(f)
    drho = np.zeros((n, n, n))
    j = np.zeros((3, n, n, n))
    sums = np.zeros(5)
    _lib().oracle_moments(_ptr(f), n, rho0, _ptr(drho), _ptr(j), _ptr(sums))
    return drho, j, sums


def init_equilibrium(u, drho=None, rho0=1.0):
    u = _f64(u)
    n = u.shape[1]
    f = np.zeros((Q, n, n, n))
    d = None if drho is None else _f64(drho, (n, n, n))
    _lib().oracle_init_equilibrium(_ptr(f), n, _ptr(u), None if d is None else _ptr(d), rho0)
    return f


def init_mrt_equilibrium(u, drho=None, rho0=1.0, w_eps=0.0, w_epsj=-475.0 / 63.0, w_xx=0.0):
    u = _f64(u)
    n = u.shape[1]
    f = np.zeros((Q, n, n, n))
    d = None if drho is None else _f64(drho, (n, n, n))
    _lib().oracle_init_mrt_equilibrium(_ptr(f), n, _ptr(u), None if d is None else _ptr(d),
                                       rho0, w_eps, w_epsj, w_xx)
    return f



def initial_pressure(u, rho0=1.0):
    """Density fluctuation consistent with a velocity field (Sec. IV.A: the
    initial pressure comes from the Poisson equation in spectral space; the
    kinetic schemes take it through the equation of state).  The
    incompressible pressure solves lap p = -rho0 d_i d_j (u_i u_j): in
    Fourier space on the integer wavevectors of the periodic grid,
    p_hat = -rho0 sum_ij k_i k_j (u_i u_j)_hat / |k|^2 (zero mean), with the
    Nyquist component of each derivative factor k_i dropped as for S and F;
    drho = p / c_s^2 = 3 p (RT = 1/3).  Returns drho[n, n, n]."""
    u = _f64(u)
    n = u.shape[1]
    k = wavenumbers(n)
    kd = np.where(np.abs(k) == n // 2, 0.0, k) if n % 2 == 0 else k
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    dz, dy, dx = np.meshgrid(kd, kd, kd, indexing="ij")
    kv = (dx, dy, dz)  # component a of u is u[a], a = 0 (x), 1 (y), 2 (z)
    k2 = kx * kx + ky * ky + kz * kz
    k2[0, 0, 0] = 1.0
    rhs = np.zeros((n, n, n), dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            rhs += kv[a] * kv[b] * np.fft.fftn(u[a] * u[b])
    p_hat = -rho0 * rhs / k2
    p_hat[0, 0, 0] = 0.0
    return 3.0 * np.real(np.fft.ifftn(p_hat))

# ----------------------------------------------------------------------------
# Consistent initial state, Sec. IV.A
# ----------------------------------------------------------------------------

def consistent_init(u, drho, method, nu, iters, rho0=1.0, mrt=None):
    """Initial LBE state consistent with a prescribed velocity field
    (Sec. IV.A: the kinetic schemes need the density fluctuation and the
    non-equilibrium part that belong to the initial velocity; the paper
    takes them from an iteration of the scheme with the velocity held at
    its initial value).

    Start from the method's equilibrium state E(drho, rho0 u) (drho = None
    for zero); then, `iters` times: one LBE step of `method` (collide then
    stream), moments (drho', j') of the new state, and
    f <- f + E(drho', rho0 u) - E(drho', j'), which puts the momentum back
    to rho0 u while keeping the density and the non-equilibrium part.  E is
    f^eq (BGK) or M^-1 m^eq (MRT), the state `init_equilibrium` /
    `init_mrt_equilibrium` build.

    Returns (f, residual): the pre-collision state and the largest change
    of drho over the last iteration (0 for iters = 0)."""
    u = _f64(u)
    m = dict(PAPER_MRT)
    if mrt:
        m.update(mrt)
    if method == "bgk":
        def E(d, j):
            return init_equilibrium(j / rho0, d, rho0)
    elif method == "mrt":
        def E(d, j):
            return init_mrt_equilibrium(j / rho0, d, rho0, m["w_eps"], m["w_epsj"], m["w_xx"])
    else:
        raise ValueError("the iteration is defined for the LBE methods")
    j0 = rho0 * u
    f = E(np.zeros(u.shape[1:]) if drho is None else _f64(drho), j0)
    d_prev = moments(f, rho0)[0]
    residual = 0.0
    for _ in range(iters):
        f = lbe_step(f, method, nu, rho0, mrt)
        d, j, _s = moments(f, rho0)
        f = f + E(d, j0) - E(d, j)
        residual = float(np.abs(d - d_prev).max())
        d_prev = d
    return f, residual


# ----------------------------------------------------------------------------
# Spectral diagnostics, Sec. III
# ----------------------------------------------------------------------------

def velocity_gradient(u):
    """G[a, b] = d_a u_b of a velocity field u[3, n, n, n] by spectral
    differentiation: the transform of d_a u_b is i kappa_a u_hat_b with
    kappa = 2 pi k / n, the Nyquist component of each derivative dropped (as
    for S and F, Sec. III, and the vorticity, Sec. IV.B).
    Returns G[3, 3, n, n, n]."""
    u = np.asarray(u, dtype=np.float64)
    n = u.shape[1]
    k1 = wavenumbers(n)
    if n % 2 == 0:
        k1 = np.where(np.abs(k1) == n // 2, 0.0, k1)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    kap = [2.0 * np.pi / n * kx, 2.0 * np.pi / n * ky, 2.0 * np.pi / n * kz]
    uh = np.fft.fftn(u, axes=(1, 2, 3))
    G = np.zeros((3, 3) + u.shape[1:])
    for a in range(3):
        for b in range(3):
            G[a, b] = np.real(np.fft.ifftn(1j * kap[a] * uh[b]))
    return G


def dugks_consistent_init(u, drho=None, nu=None, dt=0.5, rho0=1.0, tau=None):
    """Consistent initial DUGKS state for a prescribed velocity field
    (Sec. IV.A: the kinetic schemes start from the density fluctuation and
    the non-equilibrium part that belong to the initial velocity).

    The distribution is the equilibrium of Sec. II.A plus the first-order
    Chapman-Enskog non-equilibrium part of the BGK model (the collision
    Omega = (f^eq - f)/tau of Sec. II.A, tau = nu/RT): to first order in the
    gradients and lowest order in the velocity,
        f_i = f^eq_i + f1_i,
        f1_i = -(tau rho0 / RT) W_i (xi_ia xi_ib - RT delta_ab) d_a u_b,
    whose second moment is the viscous stress -rho0 nu (d_a u_b + d_b u_a)
    of a divergence-free field and whose density and momentum are zero.  The
    DUGKS tracks f~ = f - dt/2 Omega(f) (Sec. II.A), so
        f~_i = f^eq_i + (1 + dt / (2 tau)) f1_i.
    The gradient is the spectral one (velocity_gradient).  drho: the
    density fluctuation (None: 0), e.g. initial_pressure(u).
    Returns f~[19, n, n, n]."""
    u = _f64(u)
    if tau is None:
        tau = tau_dugks(nu)
    rt = 1.0 / 3.0
    f = init_equilibrium(u, drho, rho0)
    G = velocity_gradient(u)
    c, w = lattice()
    for i in range(Q):
        f1 = np.zeros(u.shape[1:])
        for a in range(3):
            for b in range(3):
                qab = c[i, a] * c[i, b] - (rt if a == b else 0.0)
                if qab != 0.0:
                    f1 += qab * G[a, b]
        f[i] += (1.0 + dt / (2.0 * tau)) * (-(tau * rho0 / rt) * w[i]) * f1
    return f


def wavenumbers(n):
    """Integer wavenumber components in numpy FFT order, -n/2 .. n/2-1."""
    return np.fft.fftfreq(n, d=1.0 / n)


def spectral_field(u):
    """u_hat(k) = DFT(u) / n^3 for each component, on all n^3 modes."""
    n = u.shape[1]
    return np.fft.fftn(np.asarray(u, dtype=np.float64), axes=(1, 2, 3)) / float(n) ** 3


def energy_spectrum(u, nu, kmax=None):
    """Shell spectrum and statistics of a velocity field u[3, n, n, n].

    E(k) = sum over modes with round(|k|) = k of 1/2 |u_hat|^2 (Sec. III,
    spectrum definition, with integer shells); K = sum of E over all modes;
    eps = 2 nu sum |kappa|^2 1/2 |u_hat|^2 with kappa = 2 pi k / n (Sec. III,
    dissipation integral).  The derivative moments behind S and F use the
    spectral derivative i kappa_a u_hat_a (the Nyquist component of each
    derivative is dropped), and S, F are the direction-averaged ratios of
    Sec. III (sum of the three third/fourth moments over the sum of the
    three matching powers of the second moments).

    Returns (E[kmax+1], dict(K, eps, S, F, u_rms, lam, eta, re_lam)).
    """
    u = np.asarray(u, dtype=np.float64)
    n = u.shape[1]
    if kmax is None:
        kmax = int(np.floor(np.sqrt(3.0) * (n // 2))) + 1
    uh = spectral_field(u)
    k1 = wavenumbers(n)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    k2 = kx * kx + ky * ky + kz * kz
    e_mode = 0.5 * np.sum(np.abs(uh) ** 2, axis=0)
    shell = np.rint(np.sqrt(k2)).astype(np.int64)
    E = np.zeros(kmax + 1)
    inside = shell <= kmax
    np.add.at(E, shell[inside], e_mode[inside])
    K = float(e_mode.sum())
    kappa2 = (2.0 * np.pi / n) ** 2 * k2
    eps = float(2.0 * nu * np.sum(kappa2 * e_mode))

    def deriv(comp, kc):
        kap = 2.0 * np.pi / n * kc
        kap = np.where(np.abs(kc) == n // 2, 0.0, kap) if n % 2 == 0 else kap
        d = np.fft.ifftn(1j * kap * uh[comp]) * float(n) ** 3
        return d.real

    num3 = den3 = num4 = den4 = 0.0
    for comp, kc in ((0, kx), (1, ky), (2, kz)):
        d = deriv(comp, kc)
        m2 = float(np.mean(d ** 2))
        num3 += float(np.mean(d ** 3))
        num4 += float(np.mean(d ** 4))
        den3 += m2 ** 1.5
        den4 += m2 ** 2
    S = num3 / den3 if den3 > 0 else 0.0
    F = num4 / den4 if den4 > 0 else 0.0
    u_rms = np.sqrt(np.mean(np.sum(u * u, axis=0)) / 3.0)
    lam = np.sqrt(15.0 * nu / eps) * u_rms if eps > 0 else np.inf
    eta = (nu ** 3 / eps) ** 0.25 if eps > 0 else np.inf
    stats = dict(K=K, eps=eps, S=S, F=F, u_rms=float(u_rms), lam=float(lam),
                 eta=float(eta), re_lam=float(u_rms * lam / nu))
    return E, stats


def vorticity(u):
    """Vorticity omega = curl u of a velocity field u[3, n, n, n] in lattice
    units (cell size 1), by spectral differentiation: omega_hat = i kappa x
    u_hat with kappa = 2 pi k / n, the Nyquist component of each derivative
    dropped as for S and F (Sec. IV.B shows the vorticity magnitude of the
    flow fields).  Returns omega[3, n, n, n]."""
    u = np.asarray(u, dtype=np.float64)
    n = u.shape[1]
    k1 = wavenumbers(n)
    if n % 2 == 0:
        k1 = np.where(np.abs(k1) == n // 2, 0.0, k1)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    kap = [2.0 * np.pi / n * kx, 2.0 * np.pi / n * ky, 2.0 * np.pi / n * kz]
    uh = np.fft.fftn(u, axes=(1, 2, 3))

    def d(comp, axis):
        return np.real(np.fft.ifftn(1j * kap[axis] * uh[comp]))

    return np.stack([d(2, 1) - d(1, 2), d(0, 2) - d(2, 0), d(1, 0) - d(0, 1)])
