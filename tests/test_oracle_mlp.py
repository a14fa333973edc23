"""Pins of the learned-corrector oracle (no GPU): finite differences, the
linear limit, Adam's closed-form first step, the exact free rotation and the
label round trip of the polar output map, and the fallback limits."""
import math

import numpy as np
import pytest

import oracle
from oracle import duffing, mlp
from paper_1404_1160_amd import synth


@pytest.mark.parametrize("n_in", [5, 6])
def test_backward_matches_central_differences(n_in):
    rng = np.random.default_rng(1)
    p = synth.mlp_init(n_in, 64, 2, seed=3).astype(np.float64)
    p += rng.normal(0, 0.05, p.size)          # non-zero biases too
    X = rng.normal(0, 1, (7, n_in))
    Y = rng.normal(0, 1, (7, 2))
    _, g = mlp.mse_loss_grad(p, X, Y)
    idx = rng.choice(p.size, 120, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(p.size)
        e[i] = h
        fd = (mlp.mse_loss_grad(p + e, X, Y)[0] - mlp.mse_loss_grad(p - e, X, Y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1e-3, abs(fd)) + 1e-10, (i, fd, g[i])


def test_activation_derivative_and_limits():
    z = np.linspace(-6, 6, 1001)
    h = 1e-6
    assert np.max(np.abs((mlp.act(z + h) - mlp.act(z - h)) / (2 * h) - mlp.act_grad(z))) < 1e-9
    assert np.all(np.abs(mlp.act(z)) < 1) and np.allclose(mlp.act(-z), -mlp.act(z))
    assert abs(mlp.act(1e8) - 1.0) < 1e-12


def test_linear_limit():
    """With weights of scale s the activation is the identity up to O(z^3), so
    the network differs from the product of its affine maps by O(s^3):
    halving s divides the difference by ~8."""
    rng = np.random.default_rng(2)
    base = [rng.normal(0, 1, (64, 5)), rng.normal(0, 1, 64), rng.normal(0, 1, (64, 64)),
            rng.normal(0, 1, 64)]
    W3, b3 = rng.normal(0, 1, (2, 64)), rng.normal(0, 1, 2)
    X = rng.normal(0, 1, (9, 5))
    errs = []
    for s in (4e-4, 2e-4, 1e-4):
        W1, b1, W2, b2 = [a * s for a in base]
        O, _ = mlp.forward(mlp.pack([W1, b1, W2, b2, W3, b3]), X)
        lin = ((X @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
        errs.append(np.max(np.abs(O - lin)))
    r = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all((r > 7.0) & (r < 9.5)), (errs, r)


def test_adam_first_step_is_signed_lr():
    """Bias correction makes the first update -lr g/(|g| + eps): a signed step."""
    rng = np.random.default_rng(3)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    g[np.abs(g) < 1e-2] = 0.5      # keep eps/|g| below 1e-6
    p1, m, v = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-2)
    assert np.allclose(p1 - p, -1e-2 * np.sign(g), rtol=2e-6, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_minimises_a_quadratic():
    target = np.linspace(-2, 3, 20)
    p = np.zeros(20)
    m = np.zeros(20)
    v = np.zeros(20)
    for t in range(1, 3001):
        p, m, v = mlp.adam_step(p, p - target, m, v, t, lr=1e-2)
    assert np.max(np.abs(p - target)) < 1e-3


def test_polar_map_identity_is_free_rotation():
    R, V, _ = synth.gaussian(100, seed=4)
    dt, eps = 0.05, 1e-3
    R1, V1 = mlp.apply_polar(R, V, dt, eps, 0.0, 0.0)
    Rx, Vx = oracle.push(R, V, dt, eps, 3, field=oracle.FIELD_ZERO)
    assert np.max(np.abs(R1 - Rx)) < 1e-12 and np.max(np.abs(V1 - Vx)) < 1e-12


def test_polar_labels_round_trip():
    rng = np.random.default_rng(5)
    R, V, _ = synth.gaussian(500, seed=5, sigma=1.5)
    dt, eps = 0.05, 1e-3
    d = rng.uniform(-3, 3, R.size)
    k = rng.uniform(-0.01, 0.01, R.size)
    R1, V1 = mlp.apply_polar(R, V, dt, eps, d, k)
    d2, k2 = mlp.polar_labels(R, V, R1, V1, dt, eps)
    assert np.max(np.abs(d2 - d)) < 1e-12 and np.max(np.abs(k2 - k)) < 1e-12
    # exact Duffing step: labels reproduce the exact end point
    Rx, Vx = duffing.solution(R, V, eps, dt)
    d3, k3 = mlp.polar_labels(R, V, Rx, Vx, dt, eps)
    R3, V3 = mlp.apply_polar(R, V, dt, eps, d3, k3)
    assert np.max(np.hypot(R3 - Rx, V3 - Vx)) < 1e-12
    # the Duffing flow advances the phase (harder spring: shorter period) and
    # changes |y| only through the orbit's shape, O(eps R^2)
    assert np.all(d3 > -1e-12) and np.max(np.abs(k3)) < 0.02


def test_scaled_polar_labels_round_trip_and_scale():
    """Amplitude-scaled map: (s, rho) = (a delta, a kappa) reproduce the same
    end point as (delta, kappa); s is the arc length at radius a.  In a
    frozen self-consistent field the phase advance of small orbits grows like
    1/a (the field jumps by 2 rho(0) at R = 0) while s stays bounded."""
    rng = np.random.default_rng(8)
    R, V, w = synth.gaussian_truncated(4000, seed=8)
    dt, eps = 0.1, 1e-3
    d = rng.uniform(-0.5, 0.5, R.size)
    k = rng.uniform(-0.01, 0.01, R.size)
    a = np.hypot(R, V)
    R1, V1 = mlp.apply_polar(R, V, dt, eps, d, k)
    R2, V2 = mlp.apply_polar(R, V, dt, eps, a * d, a * k, scaled=True)
    assert np.max(np.hypot(R1 - R2, V1 - V2)) < 1e-12
    s, rho = mlp.polar_labels(R, V, R1, V1, dt, eps, scaled=True)
    assert np.max(np.abs(s - a * d)) < 1e-12 and np.max(np.abs(rho - a * k)) < 1e-12
    # nothing moves at the origin
    R0, V0 = mlp.apply_polar(np.zeros(1), np.zeros(1), dt, eps, np.ones(1), np.ones(1), True)
    assert R0[0] == 0.0 and V0[0] == 0.0
    # frozen Poisson field of the beam, fine plain step
    nr = 1024
    rho_n, _ = oracle.deposit(R, w, nr, -5.0, 5.0)
    E, _, Qb = oracle.poisson(rho_n, nr, -5.0, 5.0)
    Rf, Vf = oracle.push(R, V, dt, eps, 400, field=oracle.FIELD_POISSON, E=E, Qb=Qb, nr=nr,
                         rmin=-5.0, rmax=5.0)
    dl, _ = mlp.polar_labels(R, V, Rf, Vf, dt, eps)
    sl, _ = mlp.polar_labels(R, V, Rf, Vf, dt, eps, scaled=True)
    small, mid = a < 0.1, (a > 0.5) & (a < 1.0)
    assert np.mean(np.abs(dl[small])) > 4 * np.mean(np.abs(dl[mid]))
    assert np.max(np.abs(sl[small])) < 2 * np.max(np.abs(sl[mid]))


def _duffing_fallback(dt, eps, K):
    return lambda R, V: oracle.push(R, V, dt, eps, K, field=oracle.FIELD_DUFFING)


def test_learned_step_fallback_limits():
    """tol = 0: every particle falls back and the step equals the plain push;
    tol = inf: none does and the step equals the network's polar map."""
    R, V, _ = synth.gaussian(300, seed=6, sigma=1.5)
    dt, eps = 0.05, 1e-3
    p = synth.mlp_init(5, 64, 2, seed=7).astype(np.float64)
    norm = mlp.Norm(mu_d=0.1, sig_d=0.05, mu_k=0.0, sig_k=1e-3)
    pot = lambda r: r ** 4 / 4
    R0, V0, fb, _ = mlp.learned_step(p, R, V, dt, eps, norm, pot, _duffing_fallback(dt, eps, 40), 0.0)
    Rp, Vp = oracle.push(R, V, dt, eps, 40, field=oracle.FIELD_DUFFING)
    assert fb.all() and np.array_equal(R0, Rp) and np.array_equal(V0, Vp)
    R1, V1, fb, _ = mlp.learned_step(p, R, V, dt, eps, norm, pot, _duffing_fallback(dt, eps, 40),
                                     math.inf)
    d, k = mlp.predict(p, R, V, dt, eps, norm)
    Rq, Vq = mlp.apply_polar(R, V, dt, eps, d, k)
    assert not fb.any() and np.array_equal(R1, Rq) and np.array_equal(V1, Vq)
    # a NaN weight makes every prediction fail the check (NaN <= tol is false)
    p_bad = p.copy()
    p_bad[100] = np.nan
    R2, V2, fb, _ = mlp.learned_step(p_bad, R, V, dt, eps, norm, pot,
                                     _duffing_fallback(dt, eps, 40), 1.0)
    assert fb.all() and np.array_equal(R2, Rp)


def test_fine_labels_match_exact_step():
    """P9: training labels from the plain push at K = 800 (eps = 1e-3, dt = 0.05,
    N(0, 1.5) beam) against the exact elliptic step's polar labels: phase
    error median < 5e-7, 99th percentile < 1e-5, max < 5e-5 (the far tail,
    |y| ~ 7); amplitude error < 5e-6.  The corrector's own phase error is
    ~1e-4."""
    R, V, _ = synth.gaussian(2000, seed=9, sigma=1.5)
    dt, eps = 0.05, 1e-3
    Rf, Vf = oracle.push(R, V, dt, eps, 800, field=oracle.FIELD_DUFFING)
    Rx, Vx = duffing.solution(R, V, eps, dt)
    d, k = mlp.polar_labels(R, V, Rf, Vf, dt, eps)
    dx, kx = mlp.polar_labels(R, V, Rx, Vx, dt, eps)
    ed = np.abs(d - dx)
    assert np.median(ed) < 5e-7 and np.percentile(ed, 99) < 1e-5 and ed.max() < 5e-5, (
        np.median(ed), ed.max())
    assert np.max(np.abs(k - kx)) < 5e-6


def test_base_polar_map_agrees_with_the_rotation_form():
    """With the free rotation as the base point, the base form of the polar
    map and of its labels is the rotation form: apply_polar(y, d, k) =
    apply_polar_to(r(dt/eps) y, d, k), plain and amplitude-scaled, and the
    labels round-trip around any base point."""
    rng = np.random.default_rng(11)
    R, V, _ = synth.gaussian(500, seed=11, sigma=1.5)
    dt, eps = 0.05, 1e-3
    d = rng.uniform(-1, 1, R.size)
    k = rng.uniform(-0.01, 0.01, R.size)
    Rb, Vb = mlp.rotate(dt / eps, R, V)
    for scaled in (False, True):
        R1, V1 = mlp.apply_polar(R, V, dt, eps, d, k, scaled=scaled)
        R2, V2 = mlp.apply_polar_to(Rb, Vb, d, k, scaled=scaled)
        assert np.max(np.hypot(R1 - R2, V1 - V2)) < 1e-12
        d1, k1 = mlp.polar_labels(R, V, R1, V1, dt, eps, scaled=scaled)
        d2, k2 = mlp.polar_labels_from(Rb, Vb, R1, V1, scaled=scaled)
        assert np.max(np.abs(d1 - d2)) < 1e-12 and np.max(np.abs(k1 - k2)) < 1e-12
    # round trip around an arbitrary base point
    Rc, Vc = R + 0.1, V - 0.2
    d3, k3 = mlp.polar_labels_from(Rc, Vc, R, V)
    R3, V3 = mlp.apply_polar_to(Rc, Vc, d3, k3)
    assert np.max(np.hypot(R3 - R, V3 - V)) < 1e-12


def test_base_push_labels_are_the_plain_push_defect():
    """Around the plain K_b-substep push the labels are that push's defect
    against the exact Duffing step: they vanish with the defect and shrink
    like K_b^-2 (the plain push is second order), while the labels around the
    free rotation stay at the size of the Duffing phase advance."""
    R, V, _ = synth.gaussian(2000, seed=12, sigma=1.5)
    dt, eps = 0.05, 1e-3
    Rx, Vx = duffing.solution(R, V, eps, dt)
    size = {}
    for Kb in (100, 200):
        Rb, Vb = oracle.push(R, V, dt, eps, Kb, field=oracle.FIELD_DUFFING)
        d, k = mlp.polar_labels_from(Rb, Vb, Rx, Vx)
        size[Kb] = np.median(np.abs(d))
        R1, V1 = mlp.apply_polar_to(Rb, Vb, d, k)
        assert np.max(np.hypot(R1 - Rx, V1 - Vx)) < 1e-12
    d0, _ = mlp.polar_labels(R, V, Rx, Vx, dt, eps)
    assert 3.0 < size[100] / size[200] < 5.0, size
    assert size[100] < 1e-3 * np.median(np.abs(d0)), (size, np.median(np.abs(d0)))


def test_learned_step_with_a_base_push():
    """A network with a base push: zero outputs give exactly the base push
    (the plain K_b step), tol = 0 gives the fallback push, and a step without
    the base push is refused."""
    R, V, _ = synth.gaussian(300, seed=13, sigma=1.5)
    dt, eps, Kb = 0.05, 1e-3, 50
    p = synth.mlp_init(5, 64, 2, seed=7).astype(np.float64)
    p[-2 - 2 * 64:] = 0.0      # W3 and b3: outputs 0
    norm = mlp.Norm(mu_d=0.0, sig_d=1e-4, mu_k=0.0, sig_k=1e-5, base_K=Kb)
    assert mlp.Norm.from_array(norm.as_array()).base_K == Kb
    pot = lambda r: r ** 4 / 4
    base = _duffing_fallback(dt, eps, Kb)
    Rb, Vb = base(R, V)
    R1, V1, fb, _ = mlp.learned_step(p, R, V, dt, eps, norm, pot, _duffing_fallback(dt, eps, 40),
                                     math.inf, base_push=base)
    assert not fb.any() and np.array_equal(R1, Rb) and np.array_equal(V1, Vb)
    R2, V2, fb, _ = mlp.learned_step(p, R, V, dt, eps, norm, pot, _duffing_fallback(dt, eps, 40),
                                     0.0, base_push=base)
    Rp, Vp = oracle.push(R, V, dt, eps, 40, field=oracle.FIELD_DUFFING)
    assert fb.all() and np.array_equal(R2, Rp) and np.array_equal(V2, Vp)
    with pytest.raises(ValueError):
        mlp.learned_step(p, R, V, dt, eps, norm, pot, _duffing_fallback(dt, eps, 40), 1.0)


def test_energy_projection_returns_to_the_shell_and_keeps_the_phase():
    """One Newton step of the radial projection: from points off the Duffing
    energy shell by a relative 1e-5 the energy error falls to O(1e-10), the
    angle of y is unchanged, points on the shell stay put, and with P = 0 the
    step is Newton's for s^2 = H0 / H1 (error (dH/H)^2 / 8 at most)."""
    rng = np.random.default_rng(14)
    R, V, _ = synth.gaussian(1000, seed=14, sigma=1.5)
    eps = 1e-3
    pot = lambda r: r ** 4 / 4
    dpot = lambda r: r ** 3
    H0 = mlp.energy(R, V, eps, pot)
    f = 1.0 + rng.uniform(-1e-5, 1e-5, R.size)
    R1, V1 = R * f, V * f
    Rp, Vp = mlp.project_energy(R1, V1, H0, eps, pot, dpot)
    assert np.max(np.abs(mlp.energy(Rp, Vp, eps, pot) / H0 - 1)) < 1e-9
    assert np.max(np.abs(np.arctan2(Vp, Rp) - np.arctan2(V1, R1))) < 1e-14
    R2, V2 = mlp.project_energy(R, V, H0, eps, pot, dpot)
    assert np.max(np.abs(R2 - R)) < 1e-14 and np.max(np.abs(V2 - V)) < 1e-14
    zero = lambda r: 0.0 * r
    H0f = mlp.energy(R, V, eps, zero)
    Rz, Vz = mlp.project_energy(R * 1.01, V * 1.01, H0f, eps, zero, zero)
    s_exact = 1.0 / 1.01
    s_newton = Rz / (R * 1.01)
    d = 1.01 ** 2 - 1.0
    assert np.max(np.abs(s_newton - s_exact)) <= d * d / 8 + 1e-15


def test_learned_step_with_projection():
    """With dpotential every particle ends on its energy shell, the network's
    and the fallback's; the decisions are those without it, and the fallback
    particles keep the angle of their plain push."""
    R, V, _ = synth.gaussian(2000, seed=15, sigma=1.5)
    dt, eps, Kb = 0.05, 1e-3, 50
    p = synth.mlp_init(5, 64, 2, seed=7).astype(np.float64)
    norm = mlp.Norm(mu_d=0.0, sig_d=2e-4, mu_k=0.0, sig_k=2e-5, base_K=Kb)
    pot = lambda r: r ** 4 / 4
    dpot = lambda r: r ** 3
    base = _duffing_fallback(dt, eps, Kb)
    fbp = _duffing_fallback(dt, eps, 40)
    _, _, _, ratio = mlp.learned_step(p, R, V, dt, eps, norm, pot, fbp, math.inf, base_push=base)
    tol = float(np.median(ratio))
    Ra, Va, fa, ra = mlp.learned_step(p, R, V, dt, eps, norm, pot, fbp, tol, base_push=base)
    Rb, Vb, fb, rb = mlp.learned_step(p, R, V, dt, eps, norm, pot, fbp, tol, base_push=base,
                                      dpotential=dpot)
    assert np.array_equal(fa, fb) and np.array_equal(ra, rb) and 0.3 < fb.mean() < 0.7
    H0 = mlp.energy(R, V, eps, pot)
    # Newton from within tol of the shell: O(tol^2) off it afterwards
    after = np.abs(mlp.energy(Rb[~fb], Vb[~fb], eps, pot) / H0[~fb] - 1)
    before = np.abs(mlp.energy(Ra[~fb], Va[~fb], eps, pot) / H0[~fb] - 1)
    assert after.max() <= tol * tol, (after.max(), tol)
    assert np.median(after) < 1e-3 * np.median(before)
    # the fallback (plain K = 40) particles: on the shell to O(r^2) of their
    # own energy error r, at the angle of the plain push
    r = np.abs(mlp.energy(Ra[fb], Va[fb], eps, pot) / H0[fb] - 1)
    after_fb = np.abs(mlp.energy(Rb[fb], Vb[fb], eps, pot) / H0[fb] - 1)
    assert np.all(after_fb <= r * r + 1e-14)
    ang = np.arctan2(Vb[fb], Rb[fb]) - np.arctan2(Va[fb], Ra[fb])
    assert np.max(np.abs(np.angle(np.exp(1j * ang)))) < 1e-14
