"""Error of the FP32 (deviation-form) path against the FP64 path.

The same initial field is advanced in FP64 and FP32 boxes; at every output
the energy spectra are compared shell by shell over the resolved shells,
1 <= k <= min(n/2, n / (2 pi eta)) (kappa_max eta <= 1 with the Kolmogorov
length eta = (nu^3/eps)^(1/4) of the FP64 run, Sec. III) whose FP64 energy
is at least 1e-10 of the largest shell energy (shells below that carry no
resolved energy: the paper's spectra end near that level), together with the
relative errors of K and eps.  The run is chaotic, so the error grows in
time; the report gives the first output where the shell error exceeds a
threshold (the horizon of that threshold).
"""
import math

import numpy as np

from . import Box


def resolved_shells(n, nu, eps):
    if eps <= 0:
        return n // 2
    eta = (nu ** 3 / eps) ** 0.25
    return max(1, min(n // 2, int(math.floor(n / (2 * math.pi * eta)))))


def turnover_time(u, nu, stream=None):
    """Large-eddy turnover time t0 = K0/eps0 of a velocity field (Sec. IV.A),
    from the library's spectrum of an FP64 box initialised with it."""
    n = u.shape[1]
    b = Box(n, "mrt", "fp64", nu, stream=stream)
    try:
        b.init_velocity_field(u)
        _, st = b.energy_spectrum(n // 2)
    finally:
        b.close()
    return st["K"] / st["eps"]


def compare_fp32_fp64(u, method, nu, steps, every, threshold=1e-4, stream=None, after_horizon=None,
                      progress=None):
    """Returns a list of outputs (dict per output step) and the horizon
    (first step whose max relative shell error exceeds `threshold`, or None).
    With `after_horizon` = m the run stops m outputs after the horizon;
    `progress(rec)` is called at every output."""
    n = u.shape[1]
    b64 = Box(n, method, "fp64", nu, stream=stream)
    b32 = Box(n, method, "fp32", nu, stream=stream)
    out, horizon = [], None
    try:
        b64.init_velocity_field(u)
        b32.init_velocity_field(u)
        done = 0
        while True:
            E64, s64 = b64.energy_spectrum(n // 2)
            E32, s32 = b32.energy_spectrum(n // 2)
            kr = resolved_shells(n, nu, s64["eps"])
            ks = np.arange(1, kr + 1)
            ks = ks[E64[ks] >= 1e-10 * E64.max()]
            rel = np.abs(E32[ks] - E64[ks]) / E64[ks]
            rec = dict(step=done, shells=int(ks.max()), max_shell_rel=float(rel.max()),
                       K_rel=float(abs(s32["K"] / s64["K"] - 1)), eps_rel=float(abs(s32["eps"] / s64["eps"] - 1)),
                       S64=float(s64["S"]), S32=float(s32["S"]))
            out.append(rec)
            if progress is not None:
                progress(rec)
            if horizon is None and rec["max_shell_rel"] > threshold:
                horizon = done
            if done >= steps:
                break
            if horizon is not None and after_horizon is not None and done >= horizon + after_horizon * every:
                break
            k = min(every, steps - done)
            b64.step(k)
            b32.step(k)
            done += k
    finally:
        b64.close()
        b32.close()
    return out, horizon
