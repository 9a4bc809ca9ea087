"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.

This module holds input recipes only: velocity fields and random population
fields.  It contains none of the LBE or DUGKS arithmetic, and it imports
neither the GPU library nor the oracle.

Array conventions: velocity fields are float64 arrays of shape (3, n, n, n)
indexed [component, z, y, x]; population fields are (19, n, n, n) indexed
[q, z, y, x].  Cell (i, j, k) sits at the point (2 pi i/n, 2 pi j/n,
2 pi k/n) of a (2 pi)^3 periodic box.
"""
import numpy as np


def grid(n):
    """Cell coordinates x_i = 2 pi i / n, i = 0..n-1."""
    return 2.0 * np.pi * np.arange(n) / n


def taylor_green(n, u0=0.05):
    """Three-dimensional Taylor-Green vortex:
    u = U0 sin x cos y cos z, v = -U0 cos x sin y cos z, w = 0."""
    x = grid(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = np.zeros((3, n, n, n))
    u[0] = u0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    u[1] = -u0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    return u


def shear_wave(n, u0=1e-3, mode=1):
    """Transverse shear wave u_x = U0 sin(2 pi mode y / n), v = w = 0."""
    x = grid(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = np.zeros((3, n, n, n))
    u[0] = u0 * np.sin(mode * Y)
    return u


def uniform_flow(n, ux, uy, uz):
    u = np.zeros((3, n, n, n))
    u[0], u[1], u[2] = ux, uy, uz
    return u


def model_spectrum(k, k0=4.0):
    """Shape of the initial spectrum, E(k) proportional to k^4 exp(-2 k^2 / k0^2)."""
    k = np.asarray(k, dtype=np.float64)
    return k ** 4 * np.exp(-2.0 * k * k / (k0 * k0))


def dhit_field(n, seed, k0=4.0, u_rms=0.05):
    """Random solenoidal velocity field with the shell spectrum
    E(k) = A k^4 exp(-2 k^2/k0^2), rescaled so that u' = sqrt(<u.u>/3) = u_rms.

    Recipe: Gaussian white noise from numpy's PCG64 seeded with `seed`,
    transformed; every mode projected onto the plane normal to k (so the
    field is divergence-free); every integer shell (round |k|) rescaled to
    the model shell energy; modes with |k| >= n/2 and the k = 0 mode set to
    zero; inverse transform; global rescale to u_rms.  Phases are the white
    noise's, hence uniform and independent."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((3, n, n, n))
    uh = np.fft.fftn(noise, axes=(1, 2, 3))
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    kk = np.stack([kx, ky, kz])
    k2 = kx * kx + ky * ky + kz * kz
    safe = np.where(k2 == 0, 1.0, k2)
    kdotu = np.sum(kk * uh, axis=0)
    uh = uh - kk * (kdotu / safe)[None]
    kmag = np.sqrt(k2)
    keep = (kmag >= 0.5) & (kmag < n / 2.0)
    uh[:, ~keep] = 0.0
    shell = np.rint(kmag).astype(np.int64)
    e_mode = 0.5 * np.sum(np.abs(uh) ** 2, axis=0)
    nshell = int(shell.max()) + 1
    e_shell = np.bincount(shell.ravel(), weights=e_mode.ravel(), minlength=nshell)
    target = model_spectrum(np.arange(nshell), k0)
    scale = np.zeros(nshell)
    ok = e_shell > 0
    scale[ok] = np.sqrt(target[ok] / e_shell[ok])
    uh = uh * scale[shell][None]
    u = np.fft.ifftn(uh, axes=(1, 2, 3)).real
    cur = np.sqrt(np.mean(np.sum(u * u, axis=0)) / 3.0)
    return np.ascontiguousarray(u * (u_rms / cur))


def dhit_field_gpu(n, seed, k0=4.0, u_rms=0.05, device="cuda", as_tensor=False):
    """`dhit_field` with its transforms and scalings done on a GPU through
    PyTorch: the same white noise (numpy PCG64 seeded with `seed`), the same
    steps in the same order; the shell energies are summed on the host
    (numpy bincount, a fixed order), so the result is the same bits on every
    call and agrees with `dhit_field` to the rounding of the two FFT
    implementations.  For callers that need many large fields quickly (a
    256^3 field takes seconds on the host).  Returns a float64 numpy array,
    or with as_tensor the contiguous float64 device tensor (the work queued
    on the calling thread's current stream done)."""
    import torch
    rng = np.random.default_rng(seed)
    noise = torch.from_numpy(rng.standard_normal((3, n, n, n))).to(device)
    uh = torch.fft.fftn(noise, dim=(1, 2, 3))
    del noise
    k1 = torch.fft.fftfreq(n, d=1.0 / n, dtype=torch.float64, device=device)
    kz, ky, kx = torch.meshgrid(k1, k1, k1, indexing="ij")
    kk = torch.stack([kx, ky, kz])
    k2 = kx * kx + ky * ky + kz * kz
    safe = torch.where(k2 == 0, torch.ones_like(k2), k2)
    kdotu = torch.sum(kk * uh, dim=0)
    uh = uh - kk * (kdotu / safe)[None]
    del kk, kdotu, safe
    kmag = torch.sqrt(k2)
    keep = (kmag >= 0.5) & (kmag < n / 2.0)
    uh = uh * keep[None]
    shell = torch.round(kmag).to(torch.int64)
    e_mode = 0.5 * torch.sum(torch.abs(uh) ** 2, dim=0)
    shell_h = shell.cpu().numpy()
    nshell = int(shell_h.max()) + 1
    e_shell = np.bincount(shell_h.ravel(), weights=e_mode.cpu().numpy().ravel(), minlength=nshell)
    target = model_spectrum(np.arange(nshell), k0)
    scale = np.zeros(nshell)
    ok = e_shell > 0
    scale[ok] = np.sqrt(target[ok] / e_shell[ok])
    uh = uh * torch.from_numpy(scale).to(device)[shell][None]
    u = torch.fft.ifftn(uh, dim=(1, 2, 3)).real
    cur = np.sqrt(float(torch.mean(torch.sum(u * u, dim=0))) / 3.0)
    u = (u * (u_rms / cur)).contiguous()
    if as_tensor:
        torch.cuda.current_stream().synchronize()
        return u
    return np.ascontiguousarray(u.cpu().numpy())


def random_populations(n, seed, amplitude=1e-2):
    """Independent uniform values in [-amplitude, amplitude] for every
    population of every cell: an arbitrary (non-equilibrium) state."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amplitude, amplitude, size=(19, n, n, n))


def random_velocity(n, seed, amplitude=1e-2):
    """Independent uniform velocity components in [-amplitude, amplitude]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amplitude, amplitude, size=(3, n, n, n))


def ensemble_grids(count=64, choices=(32, 48, 64, 96), seed=0):
    """Grid sizes of a batched ensemble, drawn uniformly from `choices`."""
    rng = np.random.default_rng(seed)
    return [int(c) for c in rng.choice(np.asarray(choices), size=count)]


def stretched_widths(n, amp=(0.2, 0.3, 0.25), phase=(0.0, 0.7, 1.9)):
    """Cell widths of a smoothly stretched periodic mesh, one row per axis:
    w_i = 1 + a cos(2 pi (i + 1/2)/n + phase), so that the box length stays
    n on every axis and the widths vary by a factor (1 + a)/(1 - a)."""
    i = np.arange(n) + 0.5
    return np.stack([1.0 + a * np.cos(2.0 * np.pi * i / n + ph) for a, ph in zip(amp, phase)])


def cell_centres(w):
    """Centres of the cells of one axis with widths w: c_0 = w_0/2,
    c_i = c_{i-1} + (w_{i-1} + w_i)/2."""
    w = np.asarray(w, dtype=np.float64)
    return np.concatenate([[0.0], np.cumsum(0.5 * (w[:-1] + w[1:]))]) + 0.5 * w[0]


def shear_wave_on_mesh(widths, u0=1e-3, mode=1):
    """u_x = U0 sin(2 pi mode y / L) at the cell centres of a stretched mesh
    (L = sum of the y widths), v = w = 0."""
    widths = np.asarray(widths, dtype=np.float64)
    n = widths.shape[1]
    yc = cell_centres(widths[1])
    L = widths[1].sum()
    u = np.zeros((3, n, n, n))
    u[0] = u0 * np.sin(2.0 * np.pi * mode * yc / L)[None, :, None]
    return u
