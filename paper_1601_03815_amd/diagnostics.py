"""Statistics of decaying isotropic turbulence (Sec. III) derived from the
library's energy spectrum and its K, eps, S, F.

Lattice units: cells of unit size in a periodic box of n cells, shell k
holds the integer wavevectors with round(|k|) = k, and the physical
wavenumber of shell k is kappa_k = 2 pi k / n (the one eps is formed with).

    u'         = sqrt(<u.u>/3) = sqrt(2 K / 3)
    lambda     = sqrt(15 nu / eps) u'          transverse Taylor microscale
    Re_lambda  = u' lambda / nu
    eta        = (nu^3 / eps)^(1/4)            Kolmogorov length
    D(k)       = 2 nu kappa_k^2 E(k)           dissipation spectrum
    kappa_max eta with kappa_max = pi (the grid's largest wavenumber, k = n/2)

Normalisations of Sec. IV.A and IV.B: time in eddy-turnover units
t' = t eps0 / K0 (t0 = K0/eps0 of the initial field), velocity magnitude
|u| / u'0 and vorticity magnitude |omega| L / u'0 with L = n, the box size
in lattice units.

`DhitStatistics.record` steps a box and collects these as time series;
`normalized_slices` gives the two magnitude fields on a plane z = const;
`to_spectral_units` converts a record to the units of the paper's
pseudo-spectral runs (box 2 pi, velocities divided by the velocity scale V_s,
Sec. IV.A).
"""
import math

import numpy as np


def statistics(E, stats, nu, n):
    """Dict of the Sec. III statistics from a spectrum E[0..kmax] and the
    library's stats (K, eps, S, F) of an n^3 box at viscosity nu."""
    K, eps = float(stats["K"]), float(stats["eps"])
    up = math.sqrt(2.0 * K / 3.0)
    lam = math.sqrt(15.0 * nu / eps) * up if eps > 0 else math.inf
    eta = (nu ** 3 / eps) ** 0.25 if eps > 0 else math.inf
    kappa = 2.0 * math.pi * np.arange(len(E)) / n
    return {
        "K": K, "eps": eps, "S": float(stats["S"]), "F": float(stats["F"]),
        "u_rms": up, "lambda": lam, "re_lambda": up * lam / nu, "eta": eta,
        "kmax_eta": math.pi * eta,
        "D": 2.0 * nu * kappa ** 2 * np.asarray(E, dtype=np.float64),
    }


class DhitStatistics:
    """Time series of the Sec. III statistics of one box."""

    def __init__(self, box, nu):
        self.box, self.nu = box, nu
        self.records = []

    def sample(self, time):
        E, st = self.box.energy_spectrum()
        rec = statistics(E, st, self.nu, self.box.n)
        rec["t"] = float(time)
        rec["E"] = np.asarray(E, dtype=np.float64)
        first = self.records[0] if self.records else rec
        # eddy-turnover time of the first sample
        rec["t_prime"] = (rec["t"] - first["t"]) * first["eps"] / first["K"] if first["K"] > 0 else 0.0
        self.records.append(rec)
        return rec

    def record(self, steps, every, dt=1.0):
        """Samples now, then every `every` steps up to `steps` more steps
        (dt: time per step, for the time axis)."""
        t0 = self.box.steps * dt
        self.sample(t0)
        done = 0
        while done < steps:
            k = min(every, steps - done)
            self.box.step(k)
            done += k
            self.sample(t0 + done * dt)
        return self.records

    def series(self, key):
        return np.array([r["t"] for r in self.records]), np.array([r[key] for r in self.records])


def normalized_slices(box, u0_rms, z=None):
    """|u| / u'0 and |omega| L / u'0 (L = n) on the plane z (default n/2, the
    plane z = L/2 of the paper's figures), as two (n, n) arrays indexed [y, x].
    The velocity comes from the box's moments and the vorticity from its
    spectral curl."""
    n = box.n
    z = n // 2 if z is None else int(z)
    _d, j, _s = box.moments()
    u = j[:, z] / box.params.rho0
    w = box.vorticity()[:, z]
    return np.sqrt(np.sum(u * u, axis=0)) / u0_rms, np.sqrt(np.sum(w * w, axis=0)) * n / u0_rms


def lattice_viscosity(nu_spectral, v_s, n):
    """Viscosity in lattice units (cell size 1, box n) of a flow whose
    spectral-unit viscosity is nu_spectral (box 2 pi) at velocity scale v_s:
    lengths scale by n / (2 pi), velocities by v_s, so nu = x^2/t scales by
    v_s n / (2 pi)."""
    return nu_spectral * v_s * n / (2.0 * math.pi)


def to_spectral_units(rec, v_s, n):
    """A record of `statistics` / `DhitStatistics` (lattice units, box n) in
    the paper's spectral units (Sec. IV.A): with ls = 2 pi / n the spectral
    length of one cell, u -> u / v_s, x -> x ls, t -> t ls v_s; so
    K -> K / v_s^2, eps and D(k) -> / (ls v_s^3), lambda and eta -> x ls,
    the shell energies E[k] -> / v_s^2 (integer shells are the same in both
    systems), nu -> nu ls / v_s.  Re_lambda, kmax eta, S, F and the
    eddy-turnover time t' are dimensionless and kept."""
    ls = 2.0 * math.pi / n
    out = dict(rec)
    out["K"] = rec["K"] / v_s ** 2
    out["u_rms"] = rec["u_rms"] / v_s
    out["eps"] = rec["eps"] / (ls * v_s ** 3)
    out["lambda"] = rec["lambda"] * ls
    out["eta"] = rec["eta"] * ls
    if "D" in rec:
        out["D"] = np.asarray(rec["D"]) / (ls * v_s ** 3)
    if "E" in rec:
        out["E"] = np.asarray(rec["E"]) / v_s ** 2
    if "t" in rec:
        out["t"] = rec["t"] * ls * v_s
    if "nu" in rec:
        out["nu"] = rec["nu"] * ls / v_s
    return out
