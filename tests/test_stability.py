"""Bisection of the stability sweep (CPU, with a stand-in for the GPU runs)."""
import math

import pytest

from paper_1601_03815_amd import stability


@pytest.mark.parametrize("threshold", [3.3e-4, 1.2e-6, 7.7e-3])
def test_bisection_brackets_the_threshold(threshold):
    runs = []

    def runner(nu):
        runs.append(nu)
        return nu >= threshold

    r = stability.max_stable_re_lambda(None, "mrt", 1e-2, 1e-7, 100.0, iters=12, runner=runner)
    assert r["bounded"]
    assert r["nu_unstable"] < threshold <= r["nu_stable"]
    assert math.log(r["nu_stable"] / r["nu_unstable"]) <= math.log(1e5) / 2 ** 12 * 1.0001
    assert len(runs) == 2 + 12


def test_bisection_reports_a_lower_bound_when_nothing_blows_up():
    r = stability.max_stable_re_lambda(None, "dugks", 1e-3, 1e-8, 100.0, runner=lambda nu: True)
    assert not r["bounded"] and r["nu_stable"] == 1e-8 and r["nu_unstable"] is None


def test_bisection_rejects_an_unstable_start():
    with pytest.raises(ValueError):
        stability.max_stable_re_lambda(None, "bgk", 1e-3, 1e-8, 100.0, runner=lambda nu: False)


def test_time_steps_follow_the_cfl_numbers():
    assert stability.time_step("mrt") == 1.0 and stability.time_step("bgk") == 1.0
    assert abs(stability.time_step("dugks") * math.sqrt(2.0) - 0.9) < 1e-15
