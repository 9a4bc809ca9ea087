"""Numerical stability at high Reynolds number (Sec. IV.E).

The paper compares the largest Taylor-microscale Reynolds number at which
each scheme still runs on a fixed mesh, accuracy aside: the LBE at CFL 1
(its time step is the lattice step) against the DUGKS at CFL 0.9
(dt = 0.9 / sqrt(2)).  Here a run is stable at viscosity nu if the global
reductions stay finite over a fixed physical time from a fixed initial
field; the largest stable Re_lambda is bracketed by bisection in log nu.
Every step runs in the library's kernels; this module only drives them.

Re_lambda is that of the initial field, Re_lambda = u' lambda / nu with
u' = sqrt(2K/3) and lambda = sqrt(15 nu u'^2 / eps) (Sec. III).  For a
fixed field eps is proportional to nu, so lambda does not depend on nu and
Re_lambda is proportional to 1/nu.
"""
import math

from . import Box, NonFiniteError

CFL_LBE = 1.0
CFL_DUGKS = 0.9


def time_step(method):
    """dt of a method at the CFL numbers of Sec. IV.E (dt = CFL / sqrt(2)
    for the DUGKS, whose fastest particle moves sqrt(2) cells per unit time)."""
    return 1.0 if method in ("bgk", "mrt") else CFL_DUGKS / math.sqrt(2.0)


def re_lambda(u, nu, precision="fp64", stream=None):
    """Taylor-microscale Reynolds number of velocity field u at viscosity nu."""
    n = u.shape[1]
    with Box(n, "mrt", precision, nu, stream=stream) as b:
        b.init_velocity_field(u)
        _, st = b.energy_spectrum(n // 2)
    up = math.sqrt(2.0 * st["K"] / 3.0)
    lam = math.sqrt(15.0 * nu * up * up / st["eps"])
    return up * lam / nu


def run_stable(u, method, nu, horizon, precision="fp64", chunk=50, stream=None):
    """Advances u with `method` at viscosity nu for `horizon` time units
    (lattice units of the LBE) and reports (stable, time reached).  The run
    is unstable once a global reduction is not finite; it is checked every
    `chunk` steps."""
    n = u.shape[1]
    dt = time_step(method)
    steps = int(math.ceil(horizon / dt))
    with Box(n, method, precision, nu, dt=dt, stream=stream) as b:
        b.init_velocity_field(u)
        done = 0
        while done < steps:
            k = min(chunk, steps - done)
            b.step(k)
            try:
                b.synchronize()
            except NonFiniteError:
                return False, done * dt
            done += k
    return True, steps * dt


def max_stable_re_lambda(u, method, nu_stable, nu_unstable, horizon, iters=10, precision="fp64",
                         stream=None, runner=None):
    """Brackets the smallest stable viscosity between nu_stable (must run to
    the horizon) and nu_unstable (must blow up) by bisection in log nu and
    returns a dict with the bracket and the Re_lambda of its stable end.
    If nu_unstable turns out stable the bracket's upper Re_lambda is a lower
    bound only (`bounded` False).  `runner(nu) -> bool` replaces the GPU run
    (for tests)."""
    run = runner or (lambda nu: run_stable(u, method, nu, horizon, precision, stream=stream)[0])
    if not run(nu_stable):
        raise ValueError("nu_stable = %g is not stable" % nu_stable)
    lo, hi = nu_unstable, nu_stable  # lo: smallest nu tried; hi: known stable
    if run(lo):
        hi, bounded = lo, False
    else:
        bounded = True
        for _ in range(iters):
            mid = math.sqrt(lo * hi)
            if run(mid):
                hi = mid
            else:
                lo = mid
    out = {"method": method, "nu_stable": hi, "nu_unstable": lo if bounded else None, "bounded": bounded,
           "horizon": horizon, "dt": time_step(method)}
    if u is not None:
        rl = re_lambda(u, hi, precision, stream)
        out["re_lambda_stable"] = rl
        out["re_lambda_unstable"] = rl * hi / lo if bounded else None
    return out
