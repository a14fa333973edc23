"""Host logic of the equal-error comparison (no GPU): the refinement of the
plain sweep and the interpolated gain, on a synthetic plain family with
error = c K^-2 and throughput = r / K, where the exact equal-error point is
known in closed form."""
import math

import pytest

from paper_1404_1160_amd import compare


def _family(c=1.0, r=1e12):
    calls = []

    def run(K):
        calls.append(K)
        return {"K": K, "rms_err": c * K ** -2.0, "particle_steps_per_s": r / K}
    return run, calls


@pytest.mark.parametrize("err", [7.0e-5, 3.3e-5, 1.2e-4])
def test_interpolated_gain_matches_the_closed_form(err):
    run, calls = _family()
    plain = [run(K) for K in (25, 50, 100, 200, 400, 800)]
    n0 = len(calls)
    learned = {"rms_err": err, "particle_steps_per_s": 2.0e10}
    res = compare._equal_error_point(plain, learned, run)
    # exact: K* = err^-1/2, plain throughput 1e12 / K*
    K_star = err ** -0.5
    assert res["gain"] == pytest.approx(2.0e10 / (1e12 / K_star), rel=1e-9)
    m = res["matched"]
    assert abs(m["err"] / err - 1) <= 0.1 and len(calls) - n0 <= 4
    lo, hi = res["plain_err_bracket"]
    assert lo > err >= hi
    # against the cheapest plain run that is not worse (more accurate, so
    # slower) the gain can only look larger
    assert res["gain_vs_cheapest_not_worse"] >= res["gain"] * (1 - 1e-12)


def test_learned_error_outside_the_sweep():
    run, _ = _family()
    plain = [run(K) for K in (25, 50)]
    res = compare._equal_error_point(plain, {"rms_err": 1e-6, "particle_steps_per_s": 1e10},
                                     None)
    assert res["gain"] is None
    res = compare._equal_error_point(plain, {"rms_err": 1.0, "particle_steps_per_s": 1e10},
                                     None)
    # below the coarsest run's error: compared with that run, no interpolation
    assert res["plain_K_bracket"] == [None, 25]
    assert res["gain"] == pytest.approx(1e10 / (1e12 / 25))
