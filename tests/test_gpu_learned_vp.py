"""Learned corrector in the self-consistent (Poisson) field vs the FP64 oracle.

The network has a sixth feature, E^n(R_n); the energy check uses the
frozen-field energy H^n = |y|^2/(2 eps) + Psi^n(R) with the mesh potential;
particles that pass are deposited by the learned kernel, the others are
pushed and deposited by the plain fallback.  Training samples are
self-generated from the context's own particles (ep_mlp_collect).

Tolerances as for the Duffing corrector: 3e-4 max(|y|, 1) (BF16 inference) or
1e-4 max(|y|, 1) (FP16) for the network map, the plain-push bound 1e-6 for fallback particles and
labels (a label is checked through the state it maps to), field after a step
2e-6 max|E|.  All cases call the HIP library through its C ABI.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1404_1160_amd import (EP_FIELD_POISSON, EP_MLP_BF16, EP_MLP_FP16, EP_PUSH_LEARNED, Sim,
                                 capi, synth)

pytestmark = pytest.mark.gpu

DT, EPS, NR, RMAX = 0.1, 1e-3, 256, 5.0
NP6 = mlp.n_params(6)
POIS = dict(field=oracle.FIELD_POISSON, nr=NR, rmin=-RMAX, rmax=RMAX)


def rel_particle(Rg, Vg, Ro, Vo):
    return np.hypot(Rg - Ro, Vg - Vo) / np.maximum(np.hypot(Ro, Vo), 1.0)


def _norm(mu_d=0.05, sig_d=0.05, mu_k=0.0, sig_k=1e-3, out_map=1):
    """Amplitude-scaled output map unless out_map = 0."""
    return mlp.Norm(s_in=1.0, s_t=100.0, s_E=0.25, mu_d=mu_d, sig_d=sig_d, mu_k=mu_k, sig_k=sig_k,
                    out_map=out_map)


def _field(R, w):
    rho, _ = oracle.deposit(R, w, NR, -RMAX, RMAX)
    E, Psi, Qb = oracle.poisson(rho, NR, -RMAX, RMAX)
    return E, Psi, Qb


MAP_TOL = {EP_MLP_BF16: 3e-4, EP_MLP_FP16: 1e-4}


def _learned_sim(n, seed, p, norm, tol, K_fb, warm_steps=0, precision=EP_MLP_BF16):
    R0, V0, w = synth.gaussian_truncated(n, seed=seed)
    sim = Sim(n, n_cells=NR, substeps=4)
    sim.set_particles(R0, V0, w)
    if warm_steps:
        sim.step(DT, EPS, EP_FIELD_POISSON, warm_steps)
    capi.ep_mlp_set_weights(sim.ctx, p, norm.as_array())
    capi.ep_set_push_mode(sim.ctx, EP_PUSH_LEARNED, tol, K_fb)
    capi.ep_mlp_set_precision(sim.ctx, precision)
    return sim, w


def test_collected_labels_match_oracle():
    n, K = 20001, 64
    R0, V0, w = synth.gaussian_truncated(n, seed=41)
    norm = _norm()
    with Sim(n, n_cells=NR, substeps=4) as sim:
        sim.set_particles(R0, V0, w)
        sim.step(DT, EPS, EP_FIELD_POISSON, 2)
        capi.ep_mlp_set_weights(sim.ctx, synth.mlp_init(6, 64, 2, seed=3), norm.as_array())
        count = capi.ep_mlp_collect(sim.ctx, DT, EPS, K, first=3, stride=7, reset=True)
        X, Y = capi.ep_mlp_get_samples(sim.ctx, 0, count)
        # a second collection appends
        assert capi.ep_mlp_collect(sim.ctx, DT, EPS, K, first=0, stride=1000) == count + 21
    idx = np.arange(3, n, 7)
    assert count == idx.size
    # the oracle's own two plain steps from the same beam give the state and
    # field the samples were collected from (the GPU state is their FP32
    # rounding, well inside the bounds below)
    R, V = oracle.run(R0, V0, w, DT, EPS, 4, 2, oracle.FIELD_POISSON, nr=NR, rmin=-RMAX,
                      rmax=RMAX)
    E, _, Qb = _field(R, w)
    Rs, Vs = R[idx], V[idx]
    Rf, Vf = oracle.push(Rs, Vs, DT, EPS, K, E=E, Qb=Qb, **POIS)
    Eg = oracle.gather(Rs, E, Qb, NR, -RMAX, RMAX)
    Xo = mlp.features(Rs, Vs, DT, EPS, norm, Egather=Eg)
    # features: 2e-6 as for the same state; the field feature E/s_E also
    # carries the field's own bound, 2e-6 max|E| (FP32 against FP64 positions)
    tol = np.full(Xo.shape[1], 2e-6)
    tol[5] += 2e-6 * np.max(np.abs(E)) / norm.s_E
    assert np.all(np.max(np.abs(X - Xo) / np.maximum(np.abs(Xo), 1.0), axis=0) <= tol)
    # each label, applied to its sample, gives the oracle's fine step
    R1, V1 = mlp.apply_polar(Rs, Vs, DT, EPS, Y[:, 0].astype(np.float64),
                             Y[:, 1].astype(np.float64), scaled=True)
    assert rel_particle(R1, V1, Rf, Vf).max() <= 1e-6
    so, ro = mlp.polar_labels(Rs, Vs, Rf, Vf, DT, EPS, scaled=True)
    assert np.max(np.abs(Y[:, 0] - so)) <= 1e-6 * max(1.0, np.max(np.abs(so)))


@pytest.mark.parametrize("precision", [EP_MLP_BF16, EP_MLP_FP16])
@pytest.mark.parametrize("out_map", [1, 0])
def test_learned_push_without_fallback_is_the_network_map(out_map, precision):
    p = synth.mlp_init(6, 64, 2, seed=9)
    norm = _norm(out_map=out_map)
    sim, w = _learned_sim(20001, 42, p, norm, 1e300, 8, precision=precision)
    R, V, _ = synth.gaussian_truncated(20001, seed=42)
    pd = p.astype(np.float64)
    for s in range(3):
        # the oracle's map from its own state, in its own field
        E, _, Qb = _field(R, w)
        Eg = oracle.gather(R, E, Qb, NR, -RMAX, RMAX)
        d, k = mlp.predict(pd, R, V, DT, EPS, norm, Egather=Eg)
        R, V = mlp.apply_polar(R, V, DT, EPS, d, k, scaled=out_map == 1)
        sim.step(DT, EPS, EP_FIELD_POISSON, 1)
        Rg, Vg = sim.particles()
        err = rel_particle(Rg, Vg, R, V)
        # per-step deviations add up (the map and the field are smooth), so
        # the bound grows with the step count
        assert err.max() <= (s + 1) * MAP_TOL[precision], (s, err.max())
        # the learned kernel deposited the new positions: its field is the one
        # a fresh context deposits from the same particles
        _, Eg_, _, _ = sim.field()
        with Sim(Rg.size, n_cells=NR) as fresh:
            fresh.set_particles(Rg, Vg, w)
            _, Ef, _, _ = fresh.field()
        assert np.max(np.abs(Eg_ - Ef)) <= 2e-6 * np.max(np.abs(Ef))
    assert sim.moments(EPS, EP_FIELD_POISSON)["n_fallback"] == 0
    sim.close()


@pytest.mark.parametrize("n", [1, 33, 63, 65, 129, 1000])
def test_learned_push_partial_waves(n):
    """Particle counts that end inside a wave (64 particles, two passes of
    32) in the self-consistent field: each particle gets its own map, and
    the deposit of the pushed particles is the field a fresh context
    deposits from them."""
    p = synth.mlp_init(6, 64, 2, seed=9)
    norm = _norm()
    sim, w = _learned_sim(n, 500 + n, p, norm, 1e300, 8, precision=EP_MLP_BF16)
    R, V, _ = synth.gaussian_truncated(n, seed=500 + n)
    E, _, Qb = _field(R, w)
    Eg = oracle.gather(R, E, Qb, NR, -RMAX, RMAX)
    d, k = mlp.predict(p.astype(np.float64), R, V, DT, EPS, norm, Egather=Eg)
    R, V = mlp.apply_polar(R, V, DT, EPS, d, k, scaled=True)
    sim.step(DT, EPS, EP_FIELD_POISSON, 1)
    Rg, Vg = sim.particles()
    assert rel_particle(Rg, Vg, R, V).max() <= MAP_TOL[EP_MLP_BF16]
    _, Eg_, _, _ = sim.field()
    with Sim(Rg.size, n_cells=NR) as fresh:
        fresh.set_particles(Rg, Vg, w)
        _, Ef, _, _ = fresh.field()
    assert np.max(np.abs(Eg_ - Ef)) <= 2e-6 * np.max(np.abs(Ef))
    assert sim.moments(EPS, EP_FIELD_POISSON)["n_fallback"] == 0
    sim.close()


def test_learned_push_all_fallback_is_the_plain_push():
    p = synth.mlp_init(6, 64, 2, seed=9)
    R0, V0, w = synth.gaussian_truncated(20001, seed=43)
    sim, _ = _learned_sim(20001, 43, p, _norm(), 0.0, 8)
    sim.step(DT, EPS, EP_FIELD_POISSON, 2)
    Rg, Vg = sim.particles()
    Ro, Vo = oracle.run(R0, V0, w, DT, EPS, 8, 2, oracle.FIELD_POISSON, nr=NR, rmin=-RMAX,
                        rmax=RMAX)
    assert rel_particle(Rg, Vg, Ro, Vo).max() <= 1e-6
    assert sim.moments(EPS, EP_FIELD_POISSON)["n_fallback"] == 2 * R0.size
    sim.close()


@pytest.mark.parametrize("precision", [EP_MLP_BF16, EP_MLP_FP16])
def test_check_decisions_agree_with_oracle(precision):
    """tol at the median drift ratio of the oracle: about half the particles
    take the network map; where the oracle's ratio is not within 20% of tol
    both sides decide alike (the map is applied in FP32 on the GPU)."""
    n, K_fb = 20001, 16
    p = synth.mlp_init(6, 64, 2, seed=10)
    norm = _norm()
    R0, V0, w = synth.gaussian_truncated(n, seed=44)
    E, Psi, Qb = _field(R0, w)
    Eg = oracle.gather(R0, E, Qb, NR, -RMAX, RMAX)
    pot = lambda r: oracle.potential(r, E, Psi, Qb, NR, -RMAX, RMAX)
    plain = lambda R, V: oracle.push(R, V, DT, EPS, K_fb, E=E, Qb=Qb, **POIS)
    pd = p.astype(np.float64)
    _, _, _, ratio = mlp.learned_step(pd, R0, V0, DT, EPS, norm, pot, plain, math.inf, Egather=Eg)
    tol = float(np.median(ratio))
    Ro, Vo, fb, ratio = mlp.learned_step(pd, R0, V0, DT, EPS, norm, pot, plain, tol, Egather=Eg)
    sim, _ = _learned_sim(n, 44, p, norm, tol, K_fb, precision=precision)
    sim.step(DT, EPS, EP_FIELD_POISSON, 1)
    Rg, Vg = sim.particles()
    nfb = sim.moments(EPS, EP_FIELD_POISSON)["n_fallback"]
    sim.close()
    clear = np.abs(ratio / tol - 1.0) > 0.2
    assert 0.3 < fb.mean() < 0.7 and clear.mean() > 0.5
    _check_decisions(Rg, Vg, R0, V0, Ro, Vo, fb, clear, pd, norm, pot, plain, Eg, precision)
    assert abs(nfb - fb.sum()) <= np.sum(~clear)


def test_check_decisions_with_projection_agree_with_oracle():
    """With the energy projection the check still decides on the network's
    prediction; where the oracle's ratio is clear of tol the GPU's result is
    the oracle's projected one (the fallback to the plain bound, the map to
    its bound), and the particles end on their frozen-field energy shells."""
    n, K_fb = 20001, 64
    p = synth.mlp_init(6, 64, 2, seed=10)
    norm = _norm()
    R0, V0, w = synth.gaussian_truncated(n, seed=44)
    E, Psi, Qb = _field(R0, w)
    Eg = oracle.gather(R0, E, Qb, NR, -RMAX, RMAX)
    pot = lambda r: oracle.potential(r, E, Psi, Qb, NR, -RMAX, RMAX)
    dpot = lambda r: -oracle.gather(r, E, Qb, NR, -RMAX, RMAX)
    plain = lambda R, V: oracle.push(R, V, DT, EPS, K_fb, E=E, Qb=Qb, **POIS)
    pd = p.astype(np.float64)
    _, _, _, ratio = mlp.learned_step(pd, R0, V0, DT, EPS, norm, pot, plain, math.inf, Egather=Eg)
    tol = float(np.median(ratio))
    Ro, Vo, fb, ratio = mlp.learned_step(pd, R0, V0, DT, EPS, norm, pot, plain, tol, Egather=Eg,
                                         dpotential=dpot)
    sim, _ = _learned_sim(n, 44, p, norm, tol, K_fb)
    capi.ep_mlp_set_projection(sim.ctx, True)
    sim.step(DT, EPS, EP_FIELD_POISSON, 1)
    Rg, Vg = sim.particles()
    nfb = sim.moments(EPS, EP_FIELD_POISSON)["n_fallback"]
    sim.close()
    clear = np.abs(ratio / tol - 1.0) > 0.2
    assert 0.3 < fb.mean() < 0.7 and clear.mean() > 0.5
    err = rel_particle(Rg, Vg, Ro, Vo)
    assert np.max(err[clear & fb], initial=0.0) <= 1e-6
    assert np.max(err[clear & ~fb], initial=0.0) <= MAP_TOL[EP_MLP_BF16]
    assert abs(nfb - fb.sum()) <= np.sum(~clear)
    # on the shell to O(r^2) of each result's own energy error r before the
    # projection (the map's, below tol; the plain push's, up to ~1e-3 at
    # K_fb = 64), plus the FP32 rounding of the stored state
    H = lambda a, b: mlp.energy(a, b, EPS, pot)
    H0 = H(R0, V0)
    drift = np.abs(H(Rg, Vg) / H0 - 1)
    Rp, Vp = plain(R0, V0)
    r = np.where(fb, np.abs(H(Rp, Vp) / H0 - 1), ratio)
    ok = drift <= 1e-6 + r * r
    assert np.mean(ok[clear]) >= 0.99, np.percentile((drift - r * r)[clear], 99)


def _check_decisions(Rg, Vg, R0, V0, Ro, Vo, fb, clear, pd, norm, pot, plain, Eg, precision):
    """Where the oracle's drift ratio is clear of tol the GPU took the
    oracle's branch; where it is not, either branch is valid (the GPU applies
    the map in FP32 before its FP64 check) and the GPU's result is one of the
    oracle's two outcomes: its network map within the map bound, or its plain
    push within the plain bound."""
    err = rel_particle(Rg, Vg, Ro, Vo)
    assert np.max(err[clear & fb], initial=0.0) <= 1e-6
    assert np.max(err[clear & ~fb], initial=0.0) <= MAP_TOL[precision]
    amb = ~clear
    Rm, Vm, _, _ = mlp.learned_step(pd, R0[amb], V0[amb], DT, EPS, norm, pot, plain, math.inf,
                                    Egather=Eg[amb])
    Rp, Vp = plain(R0[amb], V0[amb])
    as_map = rel_particle(Rg[amb], Vg[amb], Rm, Vm) <= MAP_TOL[precision]
    as_plain = rel_particle(Rg[amb], Vg[amb], Rp, Vp) <= 1e-6
    assert np.all(as_map | as_plain), np.flatnonzero(~(as_map | as_plain))[:10]


def test_gradients_six_inputs_match_oracle():
    rng = np.random.default_rng(45)
    batch = 1000
    X = rng.uniform(-1.5, 1.5, (batch, 6)).astype(np.float32)
    Y = np.stack([rng.normal(0.05, 0.05, batch), rng.normal(0.0, 1e-3, batch)], 1).astype(np.float32)
    norm = _norm()
    p = synth.mlp_init(6, 64, 2, seed=11)
    with Sim(16) as sim:
        capi.ep_mlp_set_weights(sim.ctx, p, norm.as_array())
        g, loss = capi.ep_mlp_grad(sim.ctx, X, Y, NP6)
    Yn = (Y.astype(np.float64) - [norm.mu_d, norm.mu_k]) / [norm.sig_d, norm.sig_k]
    loss_o, g_o = mlp.mse_loss_grad(p.astype(np.float64), X.astype(np.float64), Yn)
    assert abs(loss - loss_o) <= 1e-4 * loss_o
    for a, b in zip(mlp.unpack(g, 6), mlp.unpack(g_o, 6)):
        a = a.astype(np.float64).ravel()
        b = b.ravel()
        fro = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        assert fro <= 2.0 ** -6 and cos >= 0.9995, (fro, cos)


def test_training_on_collected_samples_matches_oracle_training():
    """Samples from three time levels of a plain run; a whole training run on
    the GPU against the FP64 oracle's run on the samples it collects itself
    from the same beam, in the same batch order (batch b of an epoch = rows
    b, b + P, ...): first- and last-epoch mean losses agree to 2%, and the
    loss falls."""
    n, batch, epochs, lr, lr_final = 24000, 256, 6, 3e-3, 1e-5
    R0, V0, w = synth.gaussian_truncated(n, seed=46)
    norm = _norm()
    p0 = synth.mlp_init(6, 64, 2, seed=12)
    with Sim(n, n_cells=NR, substeps=8) as sim:
        sim.set_particles(R0, V0, w)
        capi.ep_mlp_set_weights(sim.ctx, p0, norm.as_array())
        for lvl in range(3):
            total = capi.ep_mlp_collect(sim.ctx, DT, EPS, 32, first=lvl, stride=3, reset=lvl == 0)
            sim.step(DT, EPS, EP_FIELD_POISSON, 2)
        X, Y = capi.ep_mlp_get_samples(sim.ctx, 0, total)
        rep = capi.ep_mlp_train(sim.ctx, None, None, DT, EPS, 32, batch, epochs, lr, lr_final, 1.0,
                                field=EP_FIELD_POISSON)
        pg, normg = capi.ep_mlp_get_weights(sim.ctx, NP6)
    assert total == 3 * (n // 3)
    P = total // batch
    assert rep["steps"] == epochs * P and np.all(np.isfinite(pg))
    assert np.array_equal(normg[:3], norm.as_array()[:3])
    # the reported normalisation is that of the samples the GPU trained on
    Yg = Y.astype(np.float64)
    assert np.allclose([rep["mu_delta"], rep["mu_kappa"]], Yg[:65536].mean(0), rtol=1e-5,
                       atol=1e-9)
    assert np.allclose([rep["sig_delta"], rep["sig_kappa"]], Yg[:65536].std(0), rtol=1e-5)
    # the oracle collects its own samples the same way from the same beam:
    # at each level the particles lvl, lvl + 3, ... of its own plain run, the
    # features in its own field and the labels of a 32-substep push in it
    R, V = R0, V0
    Xs, Ys = [], []
    for lvl in range(3):
        E, _, Qb = _field(R, w)
        idx = np.arange(lvl, n, 3)
        Rs, Vs = R[idx], V[idx]
        Eg = oracle.gather(Rs, E, Qb, NR, -RMAX, RMAX)
        Xs.append(mlp.features(Rs, Vs, DT, EPS, norm, Egather=Eg))
        Rf, Vf = oracle.push(Rs, Vs, DT, EPS, 32, E=E, Qb=Qb, **POIS)
        Ys.append(np.stack(mlp.polar_labels(Rs, Vs, Rf, Vf, DT, EPS, scaled=True), 1))
        R, V = oracle.run(R, V, w, DT, EPS, 8, 2, oracle.FIELD_POISSON, nr=NR, rmin=-RMAX,
                          rmax=RMAX)
    Xd, Yd = np.concatenate(Xs), np.concatenate(Ys)
    mu, sd = Yd[:65536].mean(0), Yd[:65536].std(0)
    Yn = (Yd - mu) / sd
    q = p0.astype(np.float64)
    m = np.zeros_like(q)
    v = np.zeros_like(q)
    T = epochs * P
    losses = []
    for t in range(T):
        rows = (t % P) + P * np.arange(batch)
        a = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * t / T))
        loss, g = mlp.mse_loss_grad(q, Xd[rows], Yn[rows])
        losses.append(loss)
        q, m, v = mlp.adam_step(q, g, m, v, t + 1, a)
    first, last = np.mean(losses[:P]), np.mean(losses[-P:])
    assert abs(rep["loss_first"] - first) <= 0.02 * first
    assert abs(rep["loss_last"] - last) <= 0.02 * last
    assert last < 0.8 * first


def test_learned_vp_run_is_deterministic():
    p = synth.mlp_init(6, 64, 2, seed=13)
    norm = _norm()
    out = []
    for _ in range(2):
        sim, _ = _learned_sim(50001, 47, p, norm, 2e-3, 8, warm_steps=1)
        sim.step(DT, EPS, EP_FIELD_POISSON, 4)
        out.append(sim.particles() + (sim.field()[1], sim.moments(EPS, EP_FIELD_POISSON)["n_fallback"]))
        sim.close()
    (Ra, Va, Ea, fa), (Rb, Vb, Eb, fb) = out
    assert np.array_equal(Ra, Rb) and np.array_equal(Va, Vb) and np.array_equal(Ea, Eb)
    assert fa == fb and 0 < fa < 4 * 50001


def test_learned_vp_rejects_five_input_network():
    R0, V0, w = synth.gaussian_truncated(1000, seed=48)
    with Sim(1000, n_cells=NR) as sim:
        sim.set_particles(R0, V0, w)
        capi.ep_mlp_set_weights(sim.ctx, synth.mlp_init(5, 64, 2, seed=1), _norm().as_array())
        capi.ep_set_push_mode(sim.ctx, EP_PUSH_LEARNED, 1e-5, 8)
        with pytest.raises(capi.EtdpicError) as e:
            sim.step(DT, EPS, EP_FIELD_POISSON, 1)
        assert e.value.status == capi.EP_ENOTRAINED
        with pytest.raises(capi.EtdpicError) as e:
            capi.ep_mlp_collect(sim.ctx, DT, EPS, 8)
        assert e.value.status == capi.EP_ENOTRAINED


@pytest.fixture(scope="module")
def beam_1e8():
    """The Vlasov-Poisson beam at 1e8 particles (seed 17) and the oracle's
    field of all of them on N_r = 4096 cells."""
    n, nr = 100_000_000, 4096
    R0, V0, w = synth.gaussian_truncated(n, seed=17)
    rho, _ = oracle.deposit(R0, w, nr, -RMAX, RMAX)
    E, Psi, Qb = oracle.poisson(rho, nr, -RMAX, RMAX)
    return R0, V0, w, nr, E, Psi, Qb


@pytest.mark.parametrize("precision", [EP_MLP_BF16, EP_MLP_FP16])
def test_learned_vp_step_at_1e8_particles(beam_1e8, precision):
    """One learned step of the 1e8-particle beam (N_r = 4096, eps = 1e-3,
    dt = 0.1), in the launch configuration of the long-time learned run: the
    oracle takes the first and the last 10000 particles (ragged tail included)
    through its own learned step in its own field of the whole beam.  tol is
    the median drift ratio of that sample, so about half of the particles go
    to the fallback queue (5e7 entries).  Bounds as in the check-decision
    case; the beam's fallback fraction matches the sample's within sampling
    noise plus the share of undecidable particles."""
    R0, V0, w, nr, E, Psi, Qb = beam_1e8
    n, half, K_fb = R0.size, 10000, 16
    pois = dict(field=oracle.FIELD_POISSON, nr=nr, rmin=-RMAX, rmax=RMAX)
    idx = np.concatenate([np.arange(half), np.arange(n - half, n)])
    Rs, Vs = R0[idx], V0[idx]
    p = synth.mlp_init(6, 64, 2, seed=10)
    norm = _norm()
    pd = p.astype(np.float64)
    Eg = oracle.gather(Rs, E, Qb, nr, -RMAX, RMAX)
    pot = lambda r: oracle.potential(r, E, Psi, Qb, nr, -RMAX, RMAX)
    plain = lambda R, V: oracle.push(R, V, DT, EPS, K_fb, E=E, Qb=Qb, **pois)
    _, _, _, ratio = mlp.learned_step(pd, Rs, Vs, DT, EPS, norm, pot, plain, math.inf, Egather=Eg)
    tol = float(np.median(ratio))
    Ro, Vo, fb, ratio = mlp.learned_step(pd, Rs, Vs, DT, EPS, norm, pot, plain, tol, Egather=Eg)
    print("learned 1e8 precision=%d tol=%.3e" % (precision, tol), flush=True)
    with Sim(n, n_cells=nr, substeps=1) as sim:
        sim.set_particles(R0, V0, w)
        capi.ep_mlp_set_weights(sim.ctx, p, norm.as_array())
        capi.ep_set_push_mode(sim.ctx, EP_PUSH_LEARNED, tol, K_fb)
        capi.ep_mlp_set_precision(sim.ctx, precision)
        sim.step(DT, EPS, EP_FIELD_POISSON, 1)
        parts = [sim.particles(0, half), sim.particles(n - half, half)]
        m = sim.moments(EPS, EP_FIELD_POISSON)
    Rg = np.concatenate([q[0] for q in parts])
    Vg = np.concatenate([q[1] for q in parts])
    clear = np.abs(ratio / tol - 1.0) > 0.2
    assert 0.3 < fb.mean() < 0.7 and clear.mean() > 0.5
    _check_decisions(Rg, Vg, Rs, Vs, Ro, Vo, fb, clear, pd, norm, pot, plain, Eg, precision)
    assert m["n_nan"] == 0
    noise = 5.0 * math.sqrt(0.25 / idx.size)
    assert abs(m["n_fallback"] / n - fb.mean()) <= noise + np.mean(~clear)


@pytest.mark.parametrize("precision", [EP_MLP_BF16, EP_MLP_FP16])
def test_energy_projection_in_the_frozen_field_matches_oracle(precision):
    """With ep_mlp_set_projection the network map's particles are moved onto
    their frozen-field energy shell (P = Psi^n, P' = -E^n): the GPU matches
    the oracle's projected map after one step, and the frozen-field energy of
    almost every particle is kept to the FP32 rounding of the state (small
    orbits, where the slope test skips the projection, excepted)."""
    n = 20001
    p = synth.mlp_init(6, 64, 2, seed=9)
    norm = _norm(mu_d=0.0, sig_d=1e-3, sig_k=2e-5)
    sim, w = _learned_sim(n, 44, p, norm, 1e300, 8, precision=precision)
    capi.ep_mlp_set_projection(sim.ctx, True)
    R, V, _ = synth.gaussian_truncated(n, seed=44)
    E, Psi, Qb = _field(R, w)
    Eg = oracle.gather(R, E, Qb, NR, -RMAX, RMAX)
    pot = lambda r: oracle.potential(r, E, Psi, Qb, NR, -RMAX, RMAX)
    dpot = lambda r: -oracle.gather(r, E, Qb, NR, -RMAX, RMAX)
    Ro, Vo, f, ratio = mlp.learned_step(p.astype(np.float64), R, V, DT, EPS, norm, pot,
                                        lambda a, b: (a, b), math.inf, Egather=Eg,
                                        dpotential=dpot)
    assert not f.any()
    sim.step(DT, EPS, EP_FIELD_POISSON, 1)
    Rg, Vg = sim.particles()
    assert rel_particle(Rg, Vg, Ro, Vo).max() <= MAP_TOL[precision]
    H = lambda a, b: mlp.energy(a, b, EPS, pot)
    R32, V32 = R.astype(np.float32).astype(np.float64), V.astype(np.float32).astype(np.float64)
    # one Newton step leaves O(r^2) of the prediction's relative energy error
    # r; the FP32 state adds ~1e-7
    drift = np.abs(H(Rg, Vg) / H(R32, V32) - 1)
    assert np.mean(drift <= 1e-6 + ratio ** 2) >= 0.99, np.percentile(drift - ratio ** 2, 99)
    Rm, Vm, _, _ = mlp.learned_step(p.astype(np.float64), R, V, DT, EPS, norm, pot,
                                    lambda a, b: (a, b), math.inf, Egather=Eg)
    assert np.median(np.abs(H(Rm, Vm) / H(R, V) - 1)) > 10 * np.median(drift)
    sim.close()
