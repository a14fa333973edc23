"""GPU learned corrector vs the FP64 oracle (oracle/mlp.py).

Tolerances:
  * labels: FP64 plain push on both sides, FP32 output: |d delta| <= 2e-7,
    |d kappa| <= 1e-9 + 1e-6 |kappa|
  * gradients (BF16 MFMA products, FP32 accumulation) against the FP64 oracle
    at the same FP32 weights and inputs: per tensor relative Frobenius error
    <= 2^-6 and cosine >= 0.9995
  * learned step without fallback, for each inference operand type:
      - BF16 (default): split-BF16 weights (~2^-16) times activations
        rounded to BF16 (relative 2^-9); summed over 64 hidden units with
        weights ~0.1-0.2 this gives output errors up to ~4e-3 in o, and a
        particle's error is sig_d |d o| (scaled map) or sig_d |d o| |y|,
        ~2e-4 for sig_d = 0.05: the bound is 3e-4 max(|y|, 1);
      - FP16: layer-1 weights and features split into FP16 hi + lo (~2^-22),
        W2 and W3 rounded to FP16 (2^-12 relative); each activation carries
        ~3 FP16 roundings (2^-12 relative each: the pre-activation, the
        inverse square root, the product), so output errors up to ~1e-3 in
        o, particle errors ~5e-5: the bound is 1e-4 max(|y|, 1)
  * fallback: the plain push, per particle 1e-6 as for the plain path.
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


# Particle errors are relative to the particle's amplitude.  The plain
# (fallback) push is compared with a floor of 1e-3, as in the plain-path
# parity tests; the network map with a floor of 1, since its error bounds
# above are absolute errors of the outputs times sig_d (times |y| at most).
PLAIN_FLOOR, MAP_FLOOR = 1e-3, 1.0


def rel_particle(Rg, Vg, Ro, Vo, floor=PLAIN_FLOOR):
    return np.hypot(Rg - Ro, Vg - Vo) / np.maximum(np.hypot(Ro, Vo), floor)


def test_labels_match_oracle_plain_push():
    R, V, _ = synth.gaussian(4099, seed=14, sigma=SIG)
    K = 200
    with Sim(16) as sim:
        d, k = capi.ep_mlp_labels(sim.ctx, DT, EPS, K, R, V)
    Rf, Vf = oracle.push(R, V, DT, EPS, K, field=oracle.FIELD_DUFFING)
    do, ko = mlp.polar_labels(R, V, Rf, Vf, DT, EPS)
    assert np.max(np.abs(d - do)) <= 2e-7
    assert np.max(np.abs(k - ko) - 1e-6 * np.abs(ko)) <= 1e-9


def _batch(n, seed):
    R, V, _ = synth.gaussian(n, seed=seed, sigma=SIG)
    Rf, Vf = oracle.push(R, V, DT, EPS, 64, field=oracle.FIELD_DUFFING)
    d, k = mlp.polar_labels(R, V, Rf, Vf, DT, EPS)
    X = mlp.features(R, V, DT, EPS, mlp.Norm(s_in=SIG)).astype(np.float32)
    Y = np.stack([d, k], 1).astype(np.float32)
    return X, Y


def _norm_from(Y):
    mu = Y.astype(np.float64).mean(0)
    sd = Y.astype(np.float64).std(0)
    return mlp.Norm(s_in=SIG, mu_d=mu[0], sig_d=sd[0], mu_k=mu[1], sig_k=sd[1])


def _tensors(g):
    return dict(zip(("W1", "b1", "W2", "b2", "W3", "b3"), mlp.unpack(g, 5)))


@pytest.mark.parametrize("batch", [64, 1000])
def test_gradients_match_oracle(batch):
    X, Y = _batch(batch, seed=21)
    norm = _norm_from(Y)
    p = synth.mlp_init(5, 64, 2, seed=7)
    p[mlp.n_params(5) - 2:] = [0.3, -0.2]
    with Sim(16) as sim:
        capi.ep_mlp_set_weights(sim.ctx, p, norm.as_array())
        g, loss = capi.ep_mlp_grad(sim.ctx, X, Y, NP5)
    Yn = (Y.astype(np.float64) - [norm.mu_d, norm.mu_k]) / [norm.sig_d, norm.sig_k]
    loss_o, g_o = mlp.mse_loss_grad(p.astype(np.float64), X.astype(np.float64), Yn)
    assert abs(loss - loss_o) <= 1e-4 * loss_o
    for name, (a, b) in {k: (_tensors(g)[k], _tensors(g_o)[k]) for k in _tensors(g_o)}.items():
        a = a.astype(np.float64).ravel()
        b = b.ravel()
        fro = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        assert fro <= 2.0 ** -6 and cos >= 0.9995, (name, fro, cos)


def test_training_steps_match_oracle_adam():
    """Four Adam steps (constant step size) from the same start: the GPU's
    parameter change agrees with the FP64 oracle's."""
    n, batch, lr = 4096, 1024, 1e-3
    R, V, _ = synth.gaussian(n, seed=22, sigma=SIG)
    K = 64
    p0 = synth.mlp_init(5, 64, 2, seed=8)
    with Sim(16) as sim:
        capi.ep_mlp_set_weights(sim.ctx, p0, mlp.Norm(s_in=SIG).as_array())
        rep = capi.ep_mlp_train(sim.ctx, R, V, DT, EPS, K, batch, 1, lr, lr, SIG)
        pg, normg = capi.ep_mlp_get_weights(sim.ctx, NP5)
    assert rep["steps"] == n // batch
    # oracle: its own labels, normalisation, features and Adam
    Rf, Vf = oracle.push(R, V, DT, EPS, K, field=oracle.FIELD_DUFFING)
    d, k = mlp.polar_labels(R, V, Rf, Vf, DT, EPS)
    Y = np.stack([d, k], 1)
    mu, sd = Y.mean(0), Y.std(0)
    assert np.allclose([rep["mu_delta"], rep["mu_kappa"]], mu, rtol=1e-5, atol=1e-9)
    assert np.allclose([rep["sig_delta"], rep["sig_kappa"]], sd, rtol=1e-5)
    X = mlp.features(R.astype(np.float32).astype(np.float64), V, DT, EPS, mlp.Norm(s_in=SIG))
    Yn = (Y - mu) / sd
    p = p0.astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(n // batch):
        sl = slice(t * batch, (t + 1) * batch)
        _, g = mlp.mse_loss_grad(p, X[sl], Yn[sl])
        p, m, v = mlp.adam_step(p, g, m, v, t + 1, lr)
    dg = pg.astype(np.float64) - p0
    do = p - p0
    cos = dg @ do / (np.linalg.norm(dg) * np.linalg.norm(do))
    assert cos >= 0.99 and np.linalg.norm(dg - do) <= 0.1 * np.linalg.norm(do), cos


def _net(seed=9):
    p = synth.mlp_init(5, 64, 2, seed=seed)
    norm = mlp.Norm(s_in=SIG, mu_d=0.05, sig_d=0.05, mu_k=0.0, sig_k=1e-3)
    return p, norm


# bound of the network map's per-particle error, per inference operand type
MAP_TOL = {EP_MLP_BF16: 3e-4, EP_MLP_FP16: 1e-4}


def _learned_sim(R, V, w, p, norm, tol, K_fb, precision=EP_MLP_BF16):
    sim = Sim(R.size, substeps=1)
    sim.set_particles(R, V, w)
    capi.ep_mlp_set_weights(sim.ctx, p, norm.as_array())
    capi.ep_set_push_mode(sim.ctx, EP_PUSH_LEARNED, tol, K_fb)
    capi.ep_mlp_set_precision(sim.ctx, precision)
    return sim


@pytest.mark.parametrize("precision", [EP_MLP_BF16, EP_MLP_FP16])
@pytest.mark.parametrize("out_map", [0, 1])
def test_learned_push_without_fallback_is_the_network_map(out_map, precision):
    R0, V0, w = synth.gaussian(10001, seed=15, sigma=SIG)
    p, norm = _net()
    norm.out_map = out_map
    sim = _learned_sim(R0, V0, w, p, norm, 1e300, 8, precision)
    R, V = R0.copy(), V0.copy()
    pd = p.astype(np.float64)
    for s in range(3):
        sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
        d, k = mlp.predict(pd, R, V, DT, EPS, norm)
        R, V = mlp.apply_polar(R, V, DT, EPS, d, k, scaled=out_map == 1)
        Rg, Vg = sim.particles()
        err = rel_particle(Rg, Vg, R, V, MAP_FLOOR)
        # both sides continue from their own state: the per-step deviations
        # add up (the map is smooth), so the bound grows with the step count
        assert err.max() <= (s + 1) * MAP_TOL[precision], (s, err.max())
    assert sim.moments(EPS, EP_FIELD_DUFFING)["n_fallback"] == 0
    sim.close()


@pytest.mark.parametrize("precision", [EP_MLP_BF16, EP_MLP_FP16])
@pytest.mark.parametrize("n", [1, 31, 32, 33, 63, 64, 65, 127, 129, 1000])
def test_learned_push_partial_waves(n, precision):
    """A wave takes 64 particles, two network passes of 32 whose features and
    outputs cross between lanes l and l ^ 32: particle counts that end
    anywhere in a wave or in either pass give each particle its own map (no
    check) and, with tol = 0, each particle its own fallback."""
    R0, V0, w = synth.gaussian(n, seed=100 + n, sigma=SIG)
    p, norm = _net()
    pd = p.astype(np.float64)
    sim = _learned_sim(R0, V0, w, p, norm, 1e300, 8, precision)
    sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
    d, k = mlp.predict(pd, R0, V0, DT, EPS, norm)
    R, V = mlp.apply_polar(R0, V0, DT, EPS, d, k)
    Rg, Vg = sim.particles()
    assert rel_particle(Rg, Vg, R, V, MAP_FLOOR).max() <= MAP_TOL[precision]
    assert sim.moments(EPS, EP_FIELD_DUFFING)["n_fallback"] == 0
    sim.close()
    sim = _learned_sim(R0, V0, w, p, norm, 0.0, 16, precision)
    sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
    Rg, Vg = sim.particles()
    Ro, Vo = oracle.run(R0, V0, w, DT, EPS, 16, 1, oracle.FIELD_DUFFING)
    assert rel_particle(Rg, Vg, Ro, Vo).max() <= 1e-6
    assert sim.moments(EPS, EP_FIELD_DUFFING)["n_fallback"] == n
    sim.close()


def test_learned_push_all_fallback_is_the_plain_push():
    R0, V0, w = synth.gaussian(10001, seed=16, sigma=SIG)
    p, norm = _net()
    sim = _learned_sim(R0, V0, w, p, norm, 0.0, 16)
    sim.step(DT, EPS, EP_FIELD_DUFFING, 2)
    Rg, Vg = sim.particles()
    Ro, Vo = oracle.run(R0, V0, w, DT, EPS, 16, 2, oracle.FIELD_DUFFING)
    assert rel_particle(Rg, Vg, Ro, Vo).max() <= 1e-6
    assert sim.moments(EPS, EP_FIELD_DUFFING)["n_fallback"] == 2 * R0.size
    sim.close()


def test_nan_weight_forces_fallback():
    R0, V0, w = synth.gaussian(3001, seed=17, sigma=SIG)
    p, norm = _net()
    p[200] = np.nan
    sim = _learned_sim(R0, V0, w, p, norm, 1.0, 16)
    sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
    Rg, Vg = sim.particles()
    Ro, Vo = oracle.run(R0, V0, w, DT, EPS, 16, 1, oracle.FIELD_DUFFING)
    assert np.all(np.isfinite(Rg)) and rel_particle(Rg, Vg, Ro, Vo).max() <= 1e-6
    assert sim.moments(EPS, EP_FIELD_DUFFING)["n_fallback"] == R0.size
    sim.close()


def test_weights_outside_the_fp16_range_are_rejected():
    """With FP16 inference, a network whose pre-activations could leave the
    FP16 activation's range (|z| >= 16320) is refused with EP_EINVAL when a
    step needs it; the state is left untouched, a network in range works
    afterwards, and the BF16 inference (FP32 activations) runs the large
    network."""
    R0, V0, w = synth.gaussian(1000, seed=19, sigma=SIG)
    p, norm = _net()
    o_b2 = 64 * 5 + 64 + 64 * 64          # first layer-2 bias
    o_b1 = 64 * 5                         # first layer-1 bias
    for off in (o_b2, o_b1):
        bad = p.copy()
        bad[off] = 2.0e4
        sim = _learned_sim(R0, V0, w, bad, norm, 1e300, 8, EP_MLP_FP16)
        with pytest.raises(capi.EtdpicError) as ei:
            sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
        assert ei.value.status == capi.EP_EINVAL and "FP16" in str(ei.value)
        Rg, Vg = sim.particles()
        assert np.array_equal(Rg, R0.astype(np.float32).astype(np.float64))
        capi.ep_mlp_set_precision(sim.ctx, EP_MLP_BF16)
        sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
        capi.ep_mlp_set_precision(sim.ctx, EP_MLP_FP16)
        capi.ep_mlp_set_weights(sim.ctx, p, norm.as_array())
        sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
        sim.close()


@pytest.mark.parametrize("precision", [EP_MLP_BF16, EP_MLP_FP16])
def test_check_decisions_agree_with_oracle(precision):
    """With tol at the median drift ratio about half the particles take the
    network map and half the plain fallback; where the oracle's ratio is not
    within 20% of tol both sides decide alike."""
    R0, V0, w = synth.gaussian(20001, seed=18, sigma=SIG)
    p, norm = _net(seed=10)
    pot = lambda r: r ** 4 / 4
    plain = lambda R, V: oracle.push(R, V, DT, EPS, 16, field=oracle.FIELD_DUFFING)
    _, _, _, ratio = mlp.learned_step(p.astype(np.float64), R0, V0, DT, EPS, norm, pot, plain,
                                      math.inf)
    tol = float(np.median(ratio))
    Ro, Vo, fb, ratio = mlp.learned_step(p.astype(np.float64), R0, V0, DT, EPS, norm, pot, plain,
                                         tol)
    sim = _learned_sim(R0, V0, w, p, norm, tol, 16, precision)
    sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
    Rg, Vg = sim.particles()
    nfb = sim.moments(EPS, EP_FIELD_DUFFING)["n_fallback"]
    sim.close()
    clear = np.abs(ratio / tol - 1.0) > 0.2
    assert 0.3 < fb.mean() < 0.7 and clear.mean() > 0.5
    _check_decisions(Rg, Vg, R0, V0, Ro, Vo, fb, clear, p, norm, plain, precision)
    assert abs(nfb - fb.sum()) <= np.sum(~clear)


def _check_decisions(Rg, Vg, R0, V0, Ro, Vo, fb, clear, p, norm, plain, precision):
    """Where the oracle's drift ratio is clear of tol the GPU took the same
    branch as the oracle; where it is not (the GPU applies the map in FP32
    before its FP64 check, so either decision is valid there), its result is
    one of the oracle's two outcomes: the network map within the map bound,
    or the plain push within the plain path's bound."""
    err = rel_particle(Rg, Vg, Ro, Vo)
    assert np.max(err[clear & fb], initial=0.0) <= 1e-6
    err_map = rel_particle(Rg, Vg, Ro, Vo, MAP_FLOOR)
    assert np.max(err_map[clear & ~fb], initial=0.0) <= MAP_TOL[precision]
    amb = ~clear
    Rm, Vm, _, _ = mlp.learned_step(p.astype(np.float64), R0[amb], V0[amb], DT, EPS, norm,
                                    lambda r: r ** 4 / 4, plain, math.inf)
    Rp, Vp = plain(R0[amb], V0[amb])
    as_map = rel_particle(Rg[amb], Vg[amb], Rm, Vm, MAP_FLOOR) <= MAP_TOL[precision]
    as_plain = rel_particle(Rg[amb], Vg[amb], Rp, Vp) <= 1e-6
    assert np.all(as_map | as_plain), np.flatnonzero(~(as_map | as_plain))[:10]



@pytest.mark.parametrize("precision", [EP_MLP_BF16, EP_MLP_FP16])
def test_check_decisions_at_1e7_particles(precision):
    """The same check at the inference size of the Duffing comparison: 1e7
    particles of the evaluation beam (seed 15), K_fb = 400; the oracle takes
    the first and the last 10000 particles (ragged tail included) through its
    learned step, with tol at their median drift ratio, so about 5e6
    particles go to the fallback queue.  The beam's fallback fraction matches
    the sample's within sampling noise plus the share of undecidable
    particles."""
    n, half, K_fb = 10_000_000, 10000, 400
    R0, V0, w = synth.gaussian(n, seed=15, sigma=SIG)
    idx = np.concatenate([np.arange(half), np.arange(n - half, n)])
    Rs, Vs = R0[idx], V0[idx]
    p, norm = _net(seed=10)
    pd = p.astype(np.float64)
    pot = lambda r: r ** 4 / 4
    plain = lambda R, V: oracle.push(R, V, DT, EPS, K_fb, field=oracle.FIELD_DUFFING)
    _, _, _, ratio = mlp.learned_step(pd, Rs, Vs, DT, EPS, norm, pot, plain, math.inf)
    tol = float(np.median(ratio))
    Ro, Vo, fb, ratio = mlp.learned_step(pd, Rs, Vs, DT, EPS, norm, pot, plain, tol)
    print("learned duffing 1e7 precision=%d tol=%.3e" % (precision, tol), flush=True)
    sim = _learned_sim(R0, V0, w, p, norm, tol, K_fb, precision)
    sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
    parts = [sim.particles(0, half), sim.particles(n - half, half)]
    m = sim.moments(EPS, EP_FIELD_DUFFING)
    sim.close()
    Rg = np.concatenate([q[0] for q in parts])
    Vg = np.concatenate([q[1] for q in parts])
    clear = np.abs(ratio / tol - 1.0) > 0.2
    assert 0.3 < fb.mean() < 0.7 and clear.mean() > 0.5
    _check_decisions(Rg, Vg, Rs, Vs, Ro, Vo, fb, clear, p, norm, plain, precision)
    assert m["n_nan"] == 0
    noise = 5.0 * math.sqrt(0.25 / idx.size)
    assert abs(m["n_fallback"] / n - fb.mean()) <= noise + np.mean(~clear)

def test_training_run_matches_oracle_training():
    """A whole training run (labels, normalisation, 1024 Adam steps with the
    cosine schedule) on the GPU against the same run of the FP64 oracle: the
    first- and last-epoch mean losses agree to 2%, and the loss falls."""
    n, batch, epochs, K, lr, lr_final = 131072, 512, 4, 200, 3e-3, 1e-5
    R, V, _ = synth.gaussian(n, seed=23, sigma=SIG)
    p0 = synth.mlp_init(5, 64, 2, seed=5)
    with Sim(16) as sim:
        capi.ep_mlp_set_weights(sim.ctx, p0, mlp.Norm(s_in=SIG).as_array())
        rep = capi.ep_mlp_train(sim.ctx, R, V, DT, EPS, K, batch, epochs, lr, lr_final, SIG)
        p, norm = capi.ep_mlp_get_weights(sim.ctx, NP5)
    per = n // batch
    assert rep["steps"] == epochs * per
    assert np.all(np.isfinite(p))
    assert norm[3] == rep["mu_delta"] and norm[4] == rep["sig_delta"]
    Rf, Vf = oracle.push(R, V, DT, EPS, K, field=oracle.FIELD_DUFFING)
    d, k = mlp.polar_labels(R, V, Rf, Vf, DT, EPS)
    Y = np.stack([d, k], 1)
    mu, sd = Y[:65536].mean(0), Y[:65536].std(0)
    Yn = (Y - mu) / sd
    X = mlp.features(R, V, DT, EPS, mlp.Norm(s_in=SIG))
    q = p0.astype(np.float64)
    m = np.zeros_like(q)
    v = np.zeros_like(q)
    T = epochs * per
    losses = []
    for t in range(T):
        sl = slice((t % per) * batch, (t % per + 1) * batch)
        a = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * t / T))
        loss, g = mlp.mse_loss_grad(q, X[sl], Yn[sl])
        losses.append(loss)
        q, m, v = mlp.adam_step(q, g, m, v, t + 1, a)
    first, last = np.mean(losses[:per]), np.mean(losses[-per:])
    assert abs(rep["loss_first"] - first) <= 0.02 * first
    assert abs(rep["loss_last"] - last) <= 0.02 * last
    assert last < 0.5 * first
