"""GPU learned corrector with a base push (Duffing field) vs the FP64 oracle.

With K_b > 0 the polar map acts around the plain push of y_n with K_b
substeps instead of the free rotation (oracle/mlp.py: learned_step with
base_push, apply_polar_to, polar_labels_from), so the network predicts that
push's defect against the fine push.

Tolerances:
  * labels: the oracle starts from the FP32-rounded samples, as the GPU does,
    and both push in FP64: |d delta| <= 1e-9 + 1e-6 |delta| and the same for
    kappa (the FP32 rounding of the outputs);
  * the base push with a network whose outputs are zero: bitwise the plain
    push of K_b substeps after one step (same arithmetic, same table), and
    within the plain path's 1e-6 max(|y|, 1e-3) of the oracle;
  * the network map: as without a base (MAP_TOL of the operand type), plus the
    FP32 storage of the base state (6e-8 relative);
  * check decisions: as without a base (clear of tol: the same branch; near
    tol: one of the oracle's two outcomes).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1404_1160_amd import (EP_FIELD_DUFFING, EP_MLP_BF16, EP_MLP_FP16, EP_PUSH_LEARNED,
                                 EP_PUSH_PLAIN, Sim, capi, synth)

pytestmark = pytest.mark.gpu

DT, EPS, SIG = 0.05, 1e-3, 1.5
NP5 = mlp.n_params(5)
MAP_TOL = {EP_MLP_BF16: 3e-4, EP_MLP_FP16: 1e-4}
PLAIN_FLOOR, MAP_FLOOR = 1e-3, 1.0


def rel_particle(Rg, Vg, Ro, Vo, floor=PLAIN_FLOOR):
    return np.hypot(Rg - Ro, Vg - Vo) / np.maximum(np.hypot(Ro, Vo), floor)


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def push(R, V, K):
    return oracle.push(R, V, DT, EPS, K, field=oracle.FIELD_DUFFING)


def _net(Kb, seed=9, zero_out=False):
    p = synth.mlp_init(5, 64, 2, seed=seed)
    norm = mlp.Norm(s_in=SIG, mu_d=0.0, sig_d=2e-3, mu_k=0.0, sig_k=1e-4, base_K=Kb)
    if zero_out:
        p[NP5 - 2 - 2 * 64:] = 0.0    # W3, b3
    return p, norm


def _learned_sim(R, V, w, p, norm, tol, K_fb, precision=EP_MLP_BF16):
    sim = Sim(R.size, substeps=1)
    sim.set_particles(R, V, w)
    capi.ep_mlp_set_weights(sim.ctx, p, norm.as_array())
    capi.ep_set_push_mode(sim.ctx, EP_PUSH_LEARNED, tol, K_fb)
    capi.ep_mlp_set_precision(sim.ctx, precision)
    return sim


@pytest.mark.parametrize("Kb", [1, 100])
def test_base_labels_match_oracle(Kb):
    R, V, _ = synth.gaussian(4099, seed=31, sigma=SIG)
    K = 800
    p, norm = _net(Kb)
    with Sim(16) as sim:
        capi.ep_mlp_set_weights(sim.ctx, p, norm.as_array())
        d, k = capi.ep_mlp_labels(sim.ctx, DT, EPS, K, R, V)
    R32, V32 = f32(R), f32(V)
    Rb, Vb = push(R32, V32, Kb)
    Rf, Vf = push(R32, V32, K)
    do, ko = mlp.polar_labels_from(Rb, Vb, Rf, Vf)
    assert np.max(np.abs(d - do) - 1e-6 * np.abs(do)) <= 1e-9
    assert np.max(np.abs(k - ko) - 1e-6 * np.abs(ko)) <= 1e-9
    if Kb == 100:
        # the defect of K_b = 100 substeps is far below the Duffing phase advance
        d0, _ = mlp.polar_labels(R32, V32, Rf, Vf, DT, EPS)
        assert np.median(np.abs(do)) < 1e-3 * np.median(np.abs(d0))


def test_base_push_with_zero_outputs_is_the_plain_push():
    R0, V0, w = synth.gaussian(10001, seed=32, sigma=SIG)
    Kb = 64
    p, norm = _net(Kb, zero_out=True)
    sim = _learned_sim(R0, V0, w, p, norm, 1e300, 8)
    with Sim(R0.size, substeps=Kb) as plain:
        plain.set_particles(R0, V0, w)
        sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
        plain.step(DT, EPS, EP_FIELD_DUFFING, 1)
        Rg, Vg = sim.particles()
        Rp, Vp = plain.particles()
    assert np.array_equal(Rg, Rp) and np.array_equal(Vg, Vp)
    sim.step(DT, EPS, EP_FIELD_DUFFING, 2)
    Rg, Vg = sim.particles()
    Ro, Vo = R0, V0
    for _ in range(3):
        Ro, Vo = push(f32(Ro), f32(Vo), Kb)
    assert rel_particle(Rg, Vg, Ro, Vo).max() <= 1e-6
    assert sim.moments(EPS, EP_FIELD_DUFFING)["n_fallback"] == 0
    sim.close()


@pytest.mark.parametrize("precision", [EP_MLP_BF16, EP_MLP_FP16])
def test_base_push_map_matches_oracle(precision):
    """Three steps of the network map around the base push (no check) against
    the oracle's, each side from its own state."""
    R0, V0, w = synth.gaussian(10001, seed=33, sigma=SIG)
    Kb = 50
    p, norm = _net(Kb)
    sim = _learned_sim(R0, V0, w, p, norm, 1e300, 8, precision)
    pd = p.astype(np.float64)
    pot = lambda r: r ** 4 / 4
    fb = lambda R, V: push(R, V, 8)
    R, V = R0, V0
    for s in range(3):
        sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
        R, V, f, _ = mlp.learned_step(pd, R, V, DT, EPS, norm, pot, fb, math.inf,
                                      base_push=lambda a, b: push(a, b, Kb))
        assert not f.any()
        Rg, Vg = sim.particles()
        err = rel_particle(Rg, Vg, R, V, MAP_FLOOR)
        assert err.max() <= (s + 1) * MAP_TOL[precision], (s, err.max())
    # the map moved the particles off the base push by far more than the
    # parity error: the comparison sees the network
    Rb, Vb = R0, V0
    for _ in range(3):
        Rb, Vb = push(f32(Rb), f32(Vb), Kb)
    assert np.median(np.hypot(Rg - Rb, Vg - Vb)) > 100 * np.median(err)
    assert sim.moments(EPS, EP_FIELD_DUFFING)["n_fallback"] == 0
    sim.close()


@pytest.mark.parametrize("precision", [EP_MLP_BF16, EP_MLP_FP16])
def test_base_push_check_decisions_agree_with_oracle(precision):
    """tol at the median drift ratio of the oracle's map: where the oracle's
    ratio is clear of tol (by 20 %) the GPU takes the same branch, with the
    result of that branch; elsewhere its result is one of the two outcomes."""
    R0, V0, w = synth.gaussian(20001, seed=34, sigma=SIG)
    Kb, K_fb = 50, 16
    p, norm = _net(Kb, seed=10)
    pd = p.astype(np.float64)
    pot = lambda r: r ** 4 / 4
    plain = lambda R, V: push(R, V, K_fb)
    base = lambda R, V: push(R, V, Kb)
    _, _, _, ratio = mlp.learned_step(pd, R0, V0, DT, EPS, norm, pot, plain, math.inf,
                                      base_push=base)
    tol = float(np.median(ratio))
    Ro, Vo, fb, ratio = mlp.learned_step(pd, R0, V0, DT, EPS, norm, pot, plain, tol,
                                         base_push=base)
    sim = _learned_sim(R0, V0, w, p, norm, tol, K_fb, precision)
    sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
    Rg, Vg = sim.particles()
    nfb = sim.moments(EPS, EP_FIELD_DUFFING)["n_fallback"]
    sim.close()
    clear = np.abs(ratio / tol - 1.0) > 0.2
    assert 0.3 < fb.mean() < 0.7 and clear.mean() > 0.5
    err = rel_particle(Rg, Vg, Ro, Vo)
    assert np.max(err[clear & fb], initial=0.0) <= 1e-6
    err_map = rel_particle(Rg, Vg, Ro, Vo, MAP_FLOOR)
    assert np.max(err_map[clear & ~fb], initial=0.0) <= MAP_TOL[precision]
    amb = ~clear
    Rm, Vm, _, _ = mlp.learned_step(pd, R0[amb], V0[amb], DT, EPS, norm, pot, plain, math.inf,
                                    base_push=base)
    Rp, Vp = plain(R0[amb], V0[amb])
    as_map = rel_particle(Rg[amb], Vg[amb], Rm, Vm, MAP_FLOOR) <= MAP_TOL[precision]
    as_plain = rel_particle(Rg[amb], Vg[amb], Rp, Vp) <= 1e-6
    assert np.all(as_map | as_plain), np.flatnonzero(~(as_map | as_plain))[:10]
    assert abs(nfb - fb.sum()) <= np.sum(amb)


def test_base_training_uses_the_base_labels():
    """One epoch of training with a base push: the label normalisation the GPU
    sets is the mean and spread of the oracle's base labels (K_b = 50, K_fine
    = 800), not of the labels around the free rotation."""
    n, batch, Kb, K = 4096, 1024, 50, 800
    R, V, _ = synth.gaussian(n, seed=35, sigma=SIG)
    p0, norm = _net(Kb)
    with Sim(16) as sim:
        capi.ep_mlp_set_weights(sim.ctx, p0, norm.as_array())
        rep = capi.ep_mlp_train(sim.ctx, R, V, DT, EPS, K, batch, 1, 1e-3, 1e-3, SIG)
        _, normg = capi.ep_mlp_get_weights(sim.ctx, NP5)
    assert normg[8] == Kb
    R32, V32 = f32(R), f32(V)
    Rb, Vb = push(R32, V32, Kb)
    Rf, Vf = push(R32, V32, K)
    d, k = mlp.polar_labels_from(Rb, Vb, Rf, Vf)
    Y = np.stack([d, k], 1)
    assert np.allclose([rep["mu_delta"], rep["mu_kappa"]], Y.mean(0), rtol=1e-4, atol=1e-12)
    assert np.allclose([rep["sig_delta"], rep["sig_kappa"]], Y.std(0), rtol=1e-4)


def test_base_push_settings_are_validated():
    """K_b must be a whole number in [0, 4096], and only a 5-input (Duffing)
    network takes one; a rejected normalisation leaves the loaded network."""
    p, norm = _net(0)
    with Sim(16) as sim:
        capi.ep_mlp_set_weights(sim.ctx, p, norm.as_array())
        for bad in (-1.0, 2.5, 4097.0, float("nan")):
            a = norm.as_array()
            a[8] = bad
            with pytest.raises(capi.EtdpicError) as ei:
                capi.ep_mlp_set_weights(sim.ctx, p, a)
            assert ei.value.status == capi.EP_EINVAL
        a = norm.as_array()
        a[8] = 10.0
        p6 = synth.mlp_init(6, 64, 2, seed=3)
        with pytest.raises(capi.EtdpicError) as ei:
            capi.ep_mlp_set_weights(sim.ctx, p6, a)
        assert ei.value.status == capi.EP_EINVAL and "5-input" in str(ei.value)
        _, got = capi.ep_mlp_get_weights(sim.ctx, NP5)
        assert np.array_equal(got, norm.as_array())
        # an 8-value normalisation means no base push
        capi.ep_mlp_set_weights(sim.ctx, p, norm.as_array()[:8])
        assert capi.ep_mlp_get_weights(sim.ctx, NP5)[1][8] == 0.0
        # the projection switch takes 0 or 1 only
        assert capi.lib().ep_mlp_set_projection(sim.ctx, 2) == capi.EP_EINVAL
        assert capi.lib().ep_mlp_set_projection(sim.ctx, -1) == capi.EP_EINVAL
        capi.ep_mlp_set_projection(sim.ctx, True)
        capi.ep_mlp_set_projection(sim.ctx, False)


def test_base_push_survives_a_checkpoint(tmp_path):
    """A saved learned run with a base push resumes bit for bit."""
    R0, V0, w = synth.gaussian(5001, seed=36, sigma=SIG)
    p, norm = _net(40)
    path = str(tmp_path / "base.ckpt")
    sim = _learned_sim(R0, V0, w, p, norm, 1e-5, 400)
    sim.step(DT, EPS, EP_FIELD_DUFFING, 2)
    sim.save(path)
    sim.step(DT, EPS, EP_FIELD_DUFFING, 3)
    Ra, Va = sim.particles()
    sim.close()
    with Sim(R0.size, substeps=1) as s2:
        s2.load(path)
        assert capi.ep_mlp_get_weights(s2.ctx, NP5)[1][8] == 40
        s2.step(DT, EPS, EP_FIELD_DUFFING, 3)
        Rb, Vb = s2.particles()
    assert np.all(np.isfinite(Ra)) and np.all(np.isfinite(Va))
    assert np.array_equal(Ra, Rb) and np.array_equal(Va, Vb)


@pytest.mark.parametrize("precision", [EP_MLP_BF16, EP_MLP_FP16])
@pytest.mark.parametrize("Kb", [0, 50])
def test_energy_projection_matches_oracle(Kb, precision):
    """With ep_mlp_set_projection the particles that pass the check end on
    their Duffing energy shell (to the FP32 rounding of the stored state),
    and the GPU's projected map matches the oracle's over three steps, each
    side from its own state; without it the energy error is the map's."""
    R0, V0, w = synth.gaussian(10001, seed=37, sigma=SIG)
    p, norm = _net(Kb)
    pd = p.astype(np.float64)
    pot = lambda r: r ** 4 / 4
    dpot = lambda r: r ** 3
    fb = lambda R, V: push(R, V, 8)
    base = (lambda a, b: push(a, b, Kb)) if Kb else None
    H = lambda R, V: mlp.energy(R, V, EPS, pot)
    sim = _learned_sim(R0, V0, w, p, norm, 1e300, 8, precision)
    capi.ep_mlp_set_projection(sim.ctx, True)
    R, V = R0, V0
    for s in range(3):
        Rg0, Vg0 = sim.particles()
        sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
        R, V, f, ratio = mlp.learned_step(pd, R, V, DT, EPS, norm, pot, fb, math.inf,
                                          base_push=base, dpotential=dpot)
        Rg, Vg = sim.particles()
        err = rel_particle(Rg, Vg, R, V, MAP_FLOOR)
        assert err.max() <= (s + 1) * MAP_TOL[precision], (s, err.max())
        # one Newton step from the prediction's relative energy error r
        # leaves O(r^2); the FP32 state adds ~1e-7
        drift = np.abs(H(Rg, Vg) / H(Rg0, Vg0) - 1)
        assert np.all(drift <= 1e-6 + ratio ** 2), (s, np.max(drift - ratio ** 2))
        assert np.median(drift) < 1e-6
    assert sim.moments(EPS, EP_FIELD_DUFFING)["n_fallback"] == 0
    # the same network without the projection leaves its energy error
    capi.ep_mlp_set_projection(sim.ctx, False)
    Rg0, Vg0 = sim.particles()
    sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
    Rg, Vg = sim.particles()
    assert np.median(np.abs(H(Rg, Vg) / H(Rg0, Vg0) - 1)) > 10 * np.median(drift)
    sim.close()


def test_projection_keeps_the_check_decisions():
    """The check decides on the unprojected prediction, so the same particles
    fall back with and without the projection; with it, every particle (the
    network's and the fallback's) ends on its energy shell, and the GPU's
    projected results match the oracle's (clear decisions: the fallback to
    the plain-push bound, the network to its map bound)."""
    R0, V0, w = synth.gaussian(20001, seed=38, sigma=SIG)
    Kb, K_fb = 50, 400
    p, norm = _net(Kb, seed=10)
    pd = p.astype(np.float64)
    pot = lambda r: r ** 4 / 4
    dpot = lambda r: r ** 3
    plain = lambda a, b: push(a, b, K_fb)
    base = lambda a, b: push(a, b, Kb)
    _, _, _, ratio = mlp.learned_step(pd, R0, V0, DT, EPS, norm, pot, plain, math.inf,
                                      base_push=base)
    tol = float(np.median(ratio))
    Ro, Vo, fbo, ratio = mlp.learned_step(pd, R0, V0, DT, EPS, norm, pot, plain, tol,
                                          base_push=base, dpotential=dpot)
    out = {}
    for proj in (False, True):
        sim = _learned_sim(R0, V0, w, p, norm, tol, K_fb)
        capi.ep_mlp_set_projection(sim.ctx, proj)
        sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
        out[proj] = sim.particles() + (sim.moments(EPS, EP_FIELD_DUFFING)["n_fallback"],)
        sim.close()
    (_, _, na), (Rb, Vb, nb) = out[False], out[True]
    assert na == nb and 0.3 * R0.size < nb < 0.7 * R0.size
    clear = np.abs(ratio / tol - 1.0) > 0.2
    err = rel_particle(Rb, Vb, Ro, Vo)
    assert np.max(err[clear & fbo], initial=0.0) <= 1e-6
    assert np.max(rel_particle(Rb, Vb, Ro, Vo, MAP_FLOOR)[clear & ~fbo],
                  initial=0.0) <= MAP_TOL[EP_MLP_BF16]
    H = lambda R, V: mlp.energy(R, V, EPS, pot)
    H0 = H(R0.astype(np.float32).astype(np.float64), V0.astype(np.float32).astype(np.float64))
    assert np.percentile(np.abs(H(Rb, Vb) / H0 - 1), 99) < 1e-6
