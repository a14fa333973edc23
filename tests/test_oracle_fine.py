"""Pins of the oracle's reference RK4 solver and improved ETD scheme
(Algorithm 3.4) against closed forms, the exact Duffing solution and
invariants.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from oracle import duffing
from paper_1404_1160_amd import synth

NR, RMAX = 256, 5.0
VP = dict(nr=NR, rmin=-RMAX, rmax=RMAX)


def test_rk4_free_rotation_is_the_stability_polynomial():
    """E = 0: each RK4 step multiplies y by P(hA), A = M/eps, which for M^2 = -I
    is (1 - z^2/2 + z^4/24) I + (z - z^3/6) M, z = h/eps (textbook RK4
    stability polynomial of the linear part of eq. 3.1)."""
    R0, V0, w = synth.gaussian(200, seed=1)
    eps = 0.05
    h = oracle.fine_step(eps)
    z = h / eps
    a, b = 1 - z * z / 2 + z ** 4 / 24, z - z ** 3 / 6
    P = np.array([[a, b], [-b, a]])
    steps = 157
    Ps = np.linalg.matrix_power(P, steps)
    R, V = oracle.rk4_run(R0, V0, w, eps, h, steps, oracle.FIELD_ZERO)
    Rx, Vx = Ps @ np.stack([R0, V0])
    assert np.max(np.hypot(R - Rx, V - Vx) / np.hypot(R0, V0)) < 1e-13


def test_rk4_constant_field_and_duffing_are_fourth_order():
    R0, V0, w = synth.gaussian(200, seed=2)
    eps, t = 0.05, 0.8
    errs = []
    for steps in (400, 800):
        h = t / steps
        R, V = oracle.rk4_run(R0, V0, w, eps, h, steps, oracle.FIELD_DUFFING)
        Rx, Vx = duffing.solution(R0, V0, eps, t)
        errs.append(np.max(np.hypot(R - Rx, V - Vx)))
    assert 12 < errs[0] / errs[1] < 20, errs
    # constant field: y(t) = (eps E0, 0) + r(t/eps) (y0 - (eps E0, 0))
    E0, steps = 0.7, 500
    R, V = oracle.rk4_run(R0, V0, w, eps, t / steps, steps, oracle.FIELD_CONST, E0=E0)
    c, s = math.cos(t / eps), math.sin(t / eps)
    Rc = eps * E0 + c * (R0 - eps * E0) + s * V0
    Vc = -s * (R0 - eps * E0) + c * V0
    assert np.max(np.hypot(R - Rc, V - Vc)) < 1e-6


def test_rk4_coupled_poisson_run_is_symmetric_and_keeps_charge():
    R0, V0, w = synth.gaussian_truncated(3000, seed=3)
    eps = 0.01
    h = oracle.fine_step(eps)
    Ra, Va = oracle.rk4_run(R0, V0, w, eps, h, 60, oracle.FIELD_POISSON, **VP)
    Rb, Vb = oracle.rk4_run(-R0, -V0, w, eps, h, 60, oracle.FIELD_POISSON, **VP)
    assert np.max(np.abs(Ra + Rb)) < 1e-12 and np.max(np.abs(Va + Vb)) < 1e-12
    rho, off = oracle.deposit(Ra, w, NR, -RMAX, RMAX)
    assert off == 0 and abs(rho.sum() * (2 * RMAX / NR) - 1.0) < 1e-12
    # against the plain exponential integrator with many substeps over the
    # same time (both converge to the characteristics with the field frozen
    # per RK stage / per step respectively): close, not equal
    Rp, Vp = oracle.run(R0, V0, w, 60 * h, eps, 400, 1, oracle.FIELD_POISSON, **VP)
    assert np.sqrt(np.mean((Ra - Rp) ** 2)) < 1e-3


def test_periods_match_the_exact_duffing_period_and_the_free_rotation():
    R0, V0, w = synth.gaussian(500, seed=4)
    for eps in (0.05, 1e-3):
        _, _, T, N, un = oracle.improved_etd_step(R0, V0, w, 0.5, eps, oracle.FIELD_DUFFING)
        assert un == 0
        assert np.max(np.abs(T / duffing.period(R0, V0, eps) - 1)) < 1e-5
        _, _, T0, _, _ = oracle.improved_etd_step(R0, V0, w, 0.5, eps, oracle.FIELD_ZERO)
        assert np.max(np.abs(T0 / (2 * np.pi * eps) - 1)) < 1e-6
        # dt = N T + o, 0 <= o < T
        o = 0.5 - N * T
        assert np.all(o >= 0) and np.all(o < T) and np.all(N >= 1)


def test_improved_etd_is_accurate_for_periodic_orbits():
    """Duffing orbits are periodic, so Approximation 3.1 holds exactly and the
    scheme reduces to y(t_n + o_i) + N_i (y(t_n + o_i + T_i) - y(t_n + o_i));
    its error comes only from the period and the interpolation.  Against the
    exact elliptic solution at dt = 0.5 (the paper's macro step)."""
    R0, V0, w = synth.gaussian(400, seed=5)
    for eps in (0.05, 1e-3):
        R, V, T, N, un = oracle.improved_etd_step(R0, V0, w, 0.5, eps, oracle.FIELD_DUFFING)
        Rx, Vx = duffing.solution(R0, V0, eps, 0.5)
        err = np.hypot(R - Rx, V - Vx)
        # a relative period error dT shifts the phase by 2 pi N dT after N
        # periods; the quadratic interpolation errors at t_n + o and
        # t_n + o + T (~ z^3/10 |y|, z = h/eps = 2 pi/100) enter multiplied by N
        dT = np.abs(T / duffing.period(R0, V0, eps) - 1)
        z3 = (2 * np.pi / 100) ** 3
        bound = (2 * np.pi * (N + 1) * dT + (2 * N + 1) * z3 / 10) * np.hypot(Rx, Vx) * 1.5
        assert np.all(err <= bound), (eps, np.max(err / bound))
        assert np.median(err / np.maximum(np.hypot(Rx, Vx), 1.0)) < 2e-4


def test_improved_etd_with_given_periods():
    """In the given field the periods are constant, and Algorithm 3.4 may take
    them from a previous step.  With the exact elliptic periods given, the
    period term of the error bound above vanishes and only the
    interpolation term is left; with the step's own searched periods given,
    the step is the one that searches them, bit for bit; and a second step
    that reuses the first step's periods stays within the bound of two steps
    against the exact solution."""
    R0, V0, w = synth.gaussian(400, seed=6)
    for eps in (0.05, 1e-3):
        Tx = duffing.period(R0, V0, eps)
        R, V, T, N, un = oracle.improved_etd_step(R0, V0, w, 0.5, eps, oracle.FIELD_DUFFING,
                                                  T=Tx)
        assert un == 0 and np.array_equal(T, Tx)
        Rx, Vx = duffing.solution(R0, V0, eps, 0.5)
        z3 = (2 * np.pi / 100) ** 3
        bound = ((2 * N + 1) * z3 / 10) * np.hypot(Rx, Vx) * 1.5
        err = np.hypot(R - Rx, V - Vx)
        assert np.all(err <= bound), (eps, np.max(err / bound))
        Rs, Vs, Ts, Ns, _ = oracle.improved_etd_step(R0, V0, w, 0.5, eps, oracle.FIELD_DUFFING)
        Rg, Vg, Tg, Ng, _ = oracle.improved_etd_step(R0, V0, w, 0.5, eps, oracle.FIELD_DUFFING,
                                                     T=Ts)
        assert np.array_equal(Rg, Rs) and np.array_equal(Vg, Vs) and np.array_equal(Ng, Ns)
        R2, V2, _, N2, _ = oracle.improved_etd_step(Rs, Vs, w, 0.5, eps, oracle.FIELD_DUFFING,
                                                    T=Ts)
        Rx2, Vx2 = duffing.solution(R0, V0, eps, 1.0)
        dT = np.abs(Ts / Tx - 1)
        bound2 = 2 * (2 * np.pi * (N + 1) * dT + (2 * N + 1) * z3 / 10) * np.hypot(Rx2, Vx2) * 1.5
        assert np.all(np.hypot(R2 - Rx2, V2 - Vx2) <= bound2), eps


def test_improved_etd_alternative_split_at_whole_ratios():
    """Where dt / T_i is a whole number m, dt = N T_i + o_i holds with N = m,
    o_i = 0 and with N = m - 1, o_i = T_i (Algorithm 3.4, Lemma 3.3: both
    extrapolate whole periods of the same orbit).  With the exact periods given
    and dt = m T_i for some particles, the alternative split changes N_i by one
    for exactly those particles, and both results agree with the exact
    solution within the scheme's interpolation bound (the captures sit at
    other fine levels); far from whole ratios the alternative changes
    nothing."""
    R0, V0, w = synth.gaussian(300, seed=7)
    eps = 1e-3
    Tx = duffing.period(R0, V0, eps)
    m = 80
    dt = m * Tx[0]
    x = dt / Tx
    whole = np.abs(x - np.round(x)) <= 1e-9
    assert whole[0] and whole.sum() < 5
    Rs, Vs, _, Ns, _ = oracle.improved_etd_step(R0, V0, w, dt, eps, oracle.FIELD_DUFFING, T=Tx)
    Ra, Va, _, Na, _ = oracle.improved_etd_step(R0, V0, w, dt, eps, oracle.FIELD_DUFFING, T=Tx,
                                                alt_window=1e-9)
    assert np.array_equal(np.abs(Na - Ns) == 1, whole)
    assert set(Ns[whole]) | set(Na[whole]) == {m - 1, m}
    far = ~whole
    assert np.array_equal(Ra[far], Rs[far]) and np.array_equal(Va[far], Vs[far])
    Rx, Vx = duffing.solution(R0[whole], V0[whole], eps, dt)
    z3 = (2 * np.pi / 100) ** 3
    bound = ((2 * m + 1) * z3 / 10) * np.hypot(Rx, Vx) * 1.5
    for R, V in ((Rs, Vs), (Ra, Va)):
        assert np.all(np.hypot(R[whole] - Rx, V[whole] - Vx) <= bound)


def test_improved_etd_vp_step_tracks_the_reference():
    """Vlasov-Poisson beam, one macro step dt = 10 T of the improved scheme
    against the reference RK4 run over the same time: the rms radius agrees to
    the level of the scheme (the periods vary slowly)."""
    R0, V0, w = synth.gaussian_truncated(4000, seed=6)
    eps = 0.01
    dt = 20 * math.pi * eps
    R, V, T, N, un = oracle.improved_etd_step(R0, V0, w, dt, eps, oracle.FIELD_POISSON, **VP)
    assert un == 0 and np.all(N >= 8)
    h = oracle.fine_step(eps)
    Rr, Vr = oracle.rk4_run(R0, V0, w, eps, h, int(round(dt / h)), oracle.FIELD_POISSON, **VP)
    rms, rms_r = np.sqrt(np.mean(R ** 2)), np.sqrt(np.mean(Rr ** 2))
    assert abs(rms / rms_r - 1) < 2e-3
    assert np.median(np.hypot(R - Rr, V - Vr)) < 0.05


def test_classic_etd_free_rotation_and_mean_period():
    """E = 0: Algorithm 2.1 with P = 2 pi eps is the exact rotation up to the
    reference solver's error over one period, multiplied by N; the modified
    form finds P = 2 pi eps from the periods."""
    R0, V0, w = synth.gaussian(500, seed=8)
    eps, dt = 1e-3, 0.5
    c, s = math.cos(dt / eps), math.sin(dt / eps)
    for modified in (False, True):
        R, V, P, T, un = oracle.classic_etd_step(R0, V0, w, dt, eps, oracle.FIELD_ZERO, modified)
        assert un == 0 and abs(P / (2 * math.pi * eps) - 1) < 1e-6
        err = np.hypot(R - (c * R0 + s * V0), V - (-s * R0 + c * V0))
        assert np.max(err / np.hypot(R0, V0)) < 5e-4


def test_paper_claims_classic_modified_improved():
    """Section 2 and section 3: on the Duffing beam (periods differ from
    particle to particle) with dt = 0.5 >> 2 pi eps, eps = 1e-3, the classic
    scheme is inaccurate, the mean period helps, and the per-particle periods
    of Algorithm 3.4 make the step accurate (errors against the exact
    solution)."""
    R0, V0, w = synth.gaussian(1000, seed=9)
    eps, dt = 1e-3, 0.5
    Rx, Vx = duffing.solution(R0, V0, eps, dt)

    def med(R, V):
        return np.median(np.hypot(R - Rx, V - Vx))

    ec = med(*oracle.classic_etd_step(R0, V0, w, dt, eps, oracle.FIELD_DUFFING, False)[:2])
    em = med(*oracle.classic_etd_step(R0, V0, w, dt, eps, oracle.FIELD_DUFFING, True)[:2])
    ei = med(*oracle.improved_etd_step(R0, V0, w, dt, eps, oracle.FIELD_DUFFING)[:2])
    assert ei < em / 100 and em < ec, (ec, em, ei)
