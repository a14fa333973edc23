"""GPU (HIP, gfx950) vs FP64 CPU oracle: parity of the plain PIC step.

Tolerances (FP32 particle state, FP64 phase and in-register arithmetic,
exact-integer charge scan):
  * per particle, after each of 10 steps:
        |y_gpu - y_oracle|_2 / max(|y_oracle|_2, floor) <= 1e-6
    relative to the particle's own amplitude.  The floor is 1e-3 for the free
    rotation and the Duffing field, where the map is smooth and a particle's
    FP32 storage rounding stays relative to its own amplitude.  For the
    self-consistent field it is the beam size L = 1 (the paper measures
    particle errors against the size of the beam, section 1): near r = 0 that
    field jumps from -rho(0) to +rho(0) across the centre cell, so the
    discrete map stretches perturbations of small-amplitude particles
    several-fold per step, and their FP32 storage rounding is amplified in the
    oracle comparison no matter how the arithmetic is done.
  * run level, at every recorded step of a full run:
        |m_gpu - m_oracle| / |m_oracle| <= 1e-4 for rms radius and energy
  * mesh field after a deposit: |E_gpu - E_oracle| <= 2e-6 max|E|, exact
    on-mesh charge, rho to 1e-5 of its maximum (FP32 particle positions).
The oracle always starts from the seeded generator's draws and continues
from its own previous output: no GPU result is ever an oracle input.  All
cases call the HIP library through the C ABI.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1404_1160_amd import (EP_DEPOSIT_ATOMIC, EP_DEPOSIT_SORTED, EP_FIELD_DUFFING,
                                 EP_FIELD_POISSON, EP_FIELD_ZERO, Sim, capi, synth)

pytestmark = pytest.mark.gpu

TOL_PARTICLE = 1e-6
TOL_RUN = 1e-4
FLOOR = 1e-3       # smooth fields: relative to the particle's own amplitude
BEAM_SIZE = 1.0    # self-consistent field: relative to the beam size (see above)
RMAX = 5.0


def rel_particle(Rg, Vg, Ro, Vo, floor=FLOOR):
    return np.hypot(Rg - Ro, Vg - Vo) / np.maximum(np.hypot(Ro, Vo), floor)


def assert_particles(Rg, Vg, Ro, Vo, tol=TOL_PARTICLE, what="", floor=FLOOR):
    err = rel_particle(Rg, Vg, Ro, Vo, floor)
    worst = int(np.argmax(err))
    assert err[worst] <= tol, "%s: max rel err %.3e at %d (gpu %r, oracle %r)" % (
        what, err[worst], worst, (Rg[worst], Vg[worst]), (Ro[worst], Vo[worst]))


# ------------------------------------------------------------------ free rotation

def test_free_rotation_closed_form():
    R0, V0, w = synth.gaussian(10001, seed=11)
    eps, dt = 0.05, 0.1
    with Sim(R0.size, substeps=4) as sim:
        sim.set_particles(R0, V0, w)
        total = 0
        for n in (1, 6, 993, 9000):
            sim.step(dt, eps, EP_FIELD_ZERO, n)
            total += n
            R, V = sim.particles()
            t = total * dt
            Rx = R0 * np.cos(t / eps) + V0 * np.sin(t / eps)
            Vx = -R0 * np.sin(t / eps) + V0 * np.cos(t / eps)
            assert_particles(R, V, Rx, Vx, what="free rotation after %d steps" % total)
        m = sim.moments(eps, EP_FIELD_ZERO)
        assert m["n_steps"] == total
        assert math.isclose(m["t"], total * dt, rel_tol=1e-15)


# ------------------------------------------------------------------ Duffing

@pytest.mark.parametrize("K", [8, 32, 64])
def test_duffing_ten_steps_per_particle(K):
    """E = -R^3, eps = 0.05, dt = 0.1, N(0,1) beam (ragged 10001 particles).
    K >= 8: with fewer substeps the kick h*3R^2 of the tail amplitudes (|y| ~ 5)
    exceeds the state itself and the discrete map amplifies any rounding
    several-fold per step (the scheme's stability limit, not a parity issue)."""
    R0, V0, w = synth.gaussian(10001, seed=11)
    eps, dt = 0.05, 0.1
    Ro, Vo = R0.copy(), V0.copy()
    with Sim(R0.size, substeps=K) as sim:
        sim.set_particles(R0, V0, w)
        for s in range(10):
            sim.step(dt, eps, EP_FIELD_DUFFING, 1)
            Ro, Vo = oracle.push(Ro, Vo, dt, eps, K, field=oracle.FIELD_DUFFING)
            R, V = sim.particles()
            assert_particles(R, V, Ro, Vo, what="Duffing K=%d step %d" % (K, s + 1))


def test_duffing_multistep_launch_matches_single_steps():
    R0, V0, w = synth.gaussian(4099, seed=12)
    eps, dt, K = 0.05, 0.1, 16
    with Sim(R0.size, substeps=K) as a, Sim(R0.size, substeps=K) as b:
        a.set_particles(R0, V0, w)
        b.set_particles(R0, V0, w)
        a.step(dt, eps, EP_FIELD_DUFFING, 10)
        for _ in range(10):
            b.step(dt, eps, EP_FIELD_DUFFING, 1)
        Ra, Va = a.particles()
        Rb, Vb = b.particles()
        Ro, Vo = oracle.run(R0, V0, w, dt, eps, K, 10, oracle.FIELD_DUFFING)
        assert_particles(Ra, Va, Ro, Vo, what="10-step launch")
        assert_particles(Rb, Vb, Ro, Vo, what="10 single-step launches")


@pytest.mark.parametrize("K", [8, 32])
def test_duffing_full_run_moments(K):
    """Config: N_p = 1e4, eps = 0.05, dt = 0.1, 1000 steps: rms radius and
    energy within 1e-4 of the oracle every 100 steps."""
    R0, V0, w = synth.gaussian(10000, seed=11)
    eps, dt = 0.05, 0.1
    _, _, mom = oracle.run(R0, V0, w, dt, eps, K, 1000, oracle.FIELD_DUFFING, with_moments=True)
    with Sim(R0.size, substeps=K) as sim:
        sim.set_particles(R0, V0, w)
        for s in range(0, 1001, 100):
            if s:
                sim.step(dt, eps, EP_FIELD_DUFFING, 100)
            m = sim.moments(eps, EP_FIELD_DUFFING)
            for key, col in (("rms_radius", 1), ("energy", 2)):
                rel = abs(m[key] - mom[s, col]) / abs(mom[s, col])
                assert rel <= TOL_RUN, (K, s, key, m[key], mom[s, col])
            assert m["n_nan"] == 0


# ------------------------------------------------------------------ Poisson

def _oracle_field(R, w, nr):
    rho, off = oracle.deposit(R, w, nr, -RMAX, RMAX)
    E, Psi, Qb = oracle.poisson(rho, nr, -RMAX, RMAX)
    return rho, E, Psi, Qb, off


@pytest.mark.parametrize("nr", [256, 4096])
def test_deposit_and_solve(nr):
    R0, V0, w = synth.gaussian_truncated(200003, seed=12)
    # add edge cases: exact nodes, the mesh edges, off-mesh particles
    x = synth.nodes_exact(nr, RMAX)
    R0 = np.concatenate([R0, x[[0, 1, nr // 2, nr - 1]], [RMAX, -RMAX - 1e-3, 6.0]])
    V0 = np.concatenate([V0, np.zeros(7)])
    with Sim(R0.size, n_cells=nr) as sim:
        sim.set_particles(R0, V0, w)
        rho, E, Psi, Qb = sim.field()
        m = sim.moments(0.01, EP_FIELD_POISSON)
    # the generator's draws are FP32 values, and the state at phase 0 holds
    # them unchanged, so the oracle deposits exactly the GPU's positions
    Rh = R0.astype(np.float32).astype(np.float64)
    rho_o, E_o, Psi_o, Qb_o, off = _oracle_field(Rh, w, nr)
    assert m["n_offmesh"] == off == 3
    hr = 2 * RMAX / nr
    assert abs(hr * rho.sum() - w * (R0.size - off)) < 1e-12
    assert np.max(np.abs(rho - rho_o)) <= 1e-5 * np.max(rho_o)
    assert np.max(np.abs(E - E_o)) <= 2e-6 * np.max(np.abs(E_o))
    assert np.max(np.abs(Psi - Psi_o)) <= 2e-6 * np.max(np.abs(Psi_o))
    assert abs(Qb - Qb_o) <= 1e-9
    assert E[nr // 2] == 0.0
    # odd field on the symmetric mesh (up to the sampled asymmetry of the beam)
    assert np.all(np.sign(E[nr // 2 + 1:]) >= 0)


@pytest.mark.parametrize("deposit", [EP_DEPOSIT_ATOMIC, EP_DEPOSIT_SORTED])
def test_potential_after_field_only_solves(deposit):
    """Plain steps solve the field without its potential; the potential and
    field energy that ep_get_field and the moments then compute on demand
    belong to the current field: Psi is minus the trapezoid integral of the
    returned node field from the centre, and the moments' field energy the
    trapezoid of x E^2 over r >= 0 (properties of the solve at any state)."""
    nr = 256
    R0, V0, w = synth.gaussian_truncated(50001, seed=21)
    with Sim(R0.size, n_cells=nr, substeps=2, deposit=deposit) as sim:
        sim.set_particles(R0, V0, w)
        sim.step(0.05, 0.01, EP_FIELD_POISSON, 5)
        m = sim.moments(0.01, EP_FIELD_POISSON)
        rho, E, Psi, Qb = sim.field()
    hr = 2 * RMAX / nr
    c = nr // 2
    F = np.concatenate([[0.0], np.cumsum(hr * (E[:-1] + E[1:]) * 0.5)])
    assert np.max(np.abs(Psi + (F - F[c]))) <= 1e-12 * np.max(np.abs(F))
    x = (np.arange(nr + 1) - c) * hr
    right = slice(c, nr + 1)
    fe = np.trapezoid(x[right] * E[right] ** 2, dx=hr)
    assert abs(m["potential"] - fe) <= 1e-12 * fe
    assert E[c] == 0.0 and np.all(np.isfinite(Psi))


@pytest.mark.parametrize("K,deposit", [(1, EP_DEPOSIT_ATOMIC), (4, EP_DEPOSIT_ATOMIC),
                                       (1, EP_DEPOSIT_SORTED), (4, EP_DEPOSIT_SORTED)])
def test_poisson_ten_steps_per_particle(K, deposit):
    """VP beam, N_r = 256, eps = 0.01, dt = 0.05, ragged particle count."""
    R0, V0, w = synth.gaussian_truncated(20003, seed=12)
    eps, dt, nr = 0.01, 0.05, 256
    Ro, Vo = R0.copy(), V0.copy()
    with Sim(R0.size, n_cells=nr, substeps=K, deposit=deposit) as sim:
        sim.set_particles(R0, V0, w)
        for s in range(10):
            sim.step(dt, eps, EP_FIELD_POISSON, 1)
            rho, off = oracle.deposit(Ro, w, nr, -RMAX, RMAX)
            E, _, Qb = oracle.poisson(rho, nr, -RMAX, RMAX)
            Ro, Vo = oracle.push(Ro, Vo, dt, eps, K, field=oracle.FIELD_POISSON, E=E, Qb=Qb,
                                 nr=nr, rmin=-RMAX, rmax=RMAX)
            R, V = sim.particles()
            assert_particles(R, V, Ro, Vo, what="Poisson K=%d step %d" % (K, s + 1),
                             floor=BEAM_SIZE)


def test_poisson_full_run_moments():
    """2000 steps of the VP beam (N_r = 256, eps = 0.01, dt = 0.05, K = 4) at a
    reduced particle count: rms radius and energy within 1e-4 every 200 steps."""
    R0, V0, w = synth.gaussian_truncated(20000, seed=12)
    eps, dt, nr, K, n = 0.01, 0.05, 256, 4, 2000
    _, _, mom = oracle.run(R0, V0, w, dt, eps, K, n, oracle.FIELD_POISSON, nr=nr, rmin=-RMAX,
                           rmax=RMAX, with_moments=True)
    with Sim(R0.size, n_cells=nr, substeps=K) as sim:
        sim.set_particles(R0, V0, w)
        for s in range(0, n + 1, 200):
            if s:
                sim.step(dt, eps, EP_FIELD_POISSON, 200)
            m = sim.moments(eps, EP_FIELD_POISSON)
            for key, col in (("rms_radius", 1), ("energy", 2)):
                rel = abs(m[key] - mom[s, col]) / abs(mom[s, col])
                assert rel <= TOL_RUN, (s, key, m[key], mom[s, col])


def test_poisson_full_run_moments_at_config_size():
    """The Vlasov-Poisson configuration at its own size: N_p = 1e6, N_r = 256,
    eps = 0.01, dt = 0.05, 2000 steps, K = 1: rms radius and energy within
    1e-4 of the oracle every 250 steps."""
    R0, V0, w = synth.gaussian_truncated(1_000_000, seed=12)
    eps, dt, nr, K, n = 0.01, 0.05, 256, 1, 2000
    _, _, mom = oracle.run(R0, V0, w, dt, eps, K, n, oracle.FIELD_POISSON, nr=nr, rmin=-RMAX,
                           rmax=RMAX, with_moments=True)
    with Sim(R0.size, n_cells=nr, substeps=K) as sim:
        sim.set_particles(R0, V0, w)
        for s in range(0, n + 1, 250):
            if s:
                sim.step(dt, eps, EP_FIELD_POISSON, 250)
            m = sim.moments(eps, EP_FIELD_POISSON)
            for key, col in (("rms_radius", 1), ("energy", 2)):
                rel = abs(m[key] - mom[s, col]) / abs(mom[s, col])
                assert rel <= TOL_RUN, (s, key, m[key], mom[s, col])
            assert m["n_nan"] == 0


def test_poisson_changing_dt_and_eps_mid_run():
    R0, V0, w = synth.gaussian_truncated(5001, seed=13)
    nr, K = 256, 2
    Ro, Vo = R0.copy(), V0.copy()
    with Sim(R0.size, n_cells=nr, substeps=K) as sim:
        sim.set_particles(R0, V0, w)
        for dt, eps in [(0.05, 0.01), (0.02, 0.003), (0.1, 0.05)]:
            sim.step(dt, eps, EP_FIELD_POISSON, 1)
            rho, _ = oracle.deposit(Ro, w, nr, -RMAX, RMAX)
            E, _, Qb = oracle.poisson(rho, nr, -RMAX, RMAX)
            Ro, Vo = oracle.push(Ro, Vo, dt, eps, K, field=oracle.FIELD_POISSON, E=E, Qb=Qb,
                                 nr=nr, rmin=-RMAX, rmax=RMAX)
        R, V = sim.particles()
        assert_particles(R, V, Ro, Vo, what="dt/eps changed between steps", floor=BEAM_SIZE)


def test_deterministic_and_order_independent():
    """Integer fixed-point deposit: bitwise reproducible, and independent of the
    order in which particles are stored."""
    R0, V0, w = synth.gaussian_truncated(100001, seed=14)
    perm = np.random.default_rng(0).permutation(R0.size)
    out = []
    for order in (None, None, perm):
        R, V = (R0, V0) if order is None else (R0[order], V0[order])
        with Sim(R0.size, n_cells=4096, substeps=2) as sim:
            sim.set_particles(R, V, w)
            sim.step(0.05, 0.01, EP_FIELD_POISSON, 5)
            Rg, Vg = sim.particles()
            rho, E, _, _ = sim.field()
            if order is not None:
                inv = np.argsort(order)
                Rg, Vg = Rg[inv], Vg[inv]
            out.append((Rg, Vg, rho, E))
    for other in out[1:]:
        for a, b in zip(out[0], other):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("nr,K,n", [(256, 2, 100003), (4096, 1, 1000001), (256, 3, 5),
                                     (4096, 1, 100_000_000)])
def test_sorted_deposit_equals_atomic_bitwise(nr, K, n):
    """The sort-by-cell segmented reduction adds the same fixed-point weights
    as the LDS-privatised deposit, so particles (in their original order),
    charge, field and potential are bitwise identical, off-mesh and NaN
    particles included."""
    R0, V0, w = synth.gaussian_truncated(n, seed=19)
    if n > 10:
        R0[:4] = [6.0, -7.0, np.nan, 4.999]
    out = []
    for dep in (EP_DEPOSIT_ATOMIC, EP_DEPOSIT_SORTED):
        with Sim(n, n_cells=nr, substeps=K, deposit=dep) as sim:
            sim.set_particles(R0, V0, w)
            sim.step(0.05, 0.01, EP_FIELD_POISSON, 4)
            sim.step(0.1, 0.05, EP_FIELD_DUFFING, 1)      # order-preserving step in between
            sim.step(0.05, 0.01, EP_FIELD_POISSON, 3)
            R, V = sim.particles()
            part = sim.particles(n // 3, min(77, n - n // 3))
            rho, E, Psi, Qb = sim.field()
            m = sim.moments(0.01, EP_FIELD_POISSON)
        out.append((R, V, part[0], part[1], rho, E, Psi, np.array([Qb, m["n_offmesh"], m["n_nan"]])))
    for a, b in zip(*out):
        assert np.array_equal(a, b, equal_nan=True)


def test_small_and_degenerate_inputs():
    eps, dt, nr = 0.01, 0.05, 256
    for n in (1, 2, 3, 5, 7):
        R0, V0, w = synth.gaussian(n, seed=n)
        with Sim(64, n_cells=nr, substeps=3) as sim:
            sim.set_particles(R0, V0, w)
            sim.step(dt, eps, EP_FIELD_POISSON, 2)
            Ro, Vo = oracle.run(R0, V0, w, dt, eps, 3, 2, oracle.FIELD_POISSON, nr=nr,
                                rmin=-RMAX, rmax=RMAX)
            R, V = sim.particles()
            assert_particles(R, V, Ro, Vo, what="n=%d" % n, floor=BEAM_SIZE)
    # a particle at rest at the origin feels no field and stays there
    with Sim(4, n_cells=nr, substeps=2) as sim:
        sim.set_particles(np.zeros(1), np.zeros(1), 1.0)
        sim.step(dt, eps, EP_FIELD_POISSON, 3)
        R, V = sim.particles()
        assert R[0] == 0.0 and V[0] == 0.0
    # empty beam: steps and moments are well defined
    with Sim(4, n_cells=nr) as sim:
        sim.set_particles(np.zeros(0), np.zeros(0), 1.0)
        sim.step(dt, eps, EP_FIELD_POISSON, 2)
        m = sim.moments(eps, EP_FIELD_POISSON)
        assert m["charge"] == 0.0 and m["n_nan"] == 0


def test_off_mesh_and_nan_particles_are_counted():
    R0, V0, w = synth.gaussian_truncated(1000, seed=15)
    R0[:3] = [7.0, -8.0, 5.5]
    V0[:3] = 0.0
    R0[3] = np.nan
    with Sim(R0.size, n_cells=256, substeps=2) as sim:
        sim.set_particles(R0, V0, w)
        m = sim.moments(0.01, EP_FIELD_POISSON)
        assert m["n_nan"] == 1
        assert m["n_offmesh"] == 3
        sim.step(0.05, 0.01, EP_FIELD_POISSON, 3)
        R, V = sim.particles()
        assert np.isnan(R[3]) and np.all(np.isfinite(R[4:]))
        ok = np.isfinite(R0)
        Ro, Vo = oracle.run(R0[ok], V0[ok], w, 0.05, 0.01, 2, 3, oracle.FIELD_POISSON, nr=256,
                            rmin=-RMAX, rmax=RMAX)
        assert_particles(R[ok], V[ok], Ro, Vo, what="off-mesh particles", floor=BEAM_SIZE)


def test_invalid_step_arguments():
    with Sim(16, n_cells=256) as sim:
        with pytest.raises(capi.EtdpicError):
            sim.step(0.1, 0.1, EP_FIELD_DUFFING)   # no particles yet
        sim.set_particles(np.ones(4), np.zeros(4), 0.25)
        for dt, eps, field in [(0.0, 0.1, 1), (0.1, -1.0, 1), (0.1, 0.1, 9), (math.nan, 0.1, 1)]:
            with pytest.raises(capi.EtdpicError) as ei:
                sim.step(dt, eps, field)
            assert ei.value.status == capi.EP_EINVAL
        with pytest.raises(capi.EtdpicError):
            sim.set_particles(np.ones(17), np.ones(17), 0.1)   # over capacity


# ------------------------------------------------------------------ at full size

def full_size_parity(n, nr, eps, dt, K, n_steps, n_sample, seed, edge=False):
    """Per-particle parity at full size: the oracle runs the whole seeded beam
    itself (its own deposit, field and push of every particle, step after
    step, from its own previous state), and a sample of particles (the first
    and the last n_sample/2, so the ragged tail is included) is compared with
    the GPU run after every step, with the run's rms radius and energy.
    edge: the first particles are placed at radii around the mesh edge, so
    that their wave mixes particles that provably stay on the mesh with ones
    that may leave it (two gather paths in one wave)."""
    R0, V0, w = synth.gaussian_truncated(n, seed=seed)
    if edge:
        radii = np.array([4.90, 4.95, 4.98, 4.995, 5.0, 5.01, 5.05, 5.2, 3.0, 0.5])
        ang = np.linspace(0.1, 6.0, radii.size)
        R0[:radii.size] = radii * np.cos(ang)
        V0[:radii.size] = radii * np.sin(ang)
    half = n_sample // 2
    ranges = [(0, half), (n - half, half)]
    idx = np.concatenate([np.arange(a, a + c) for a, c in ranges])
    worst = 0.0
    with Sim(n, n_cells=nr, substeps=K) as sim:
        sim.set_particles(R0, V0, w)
        Ro, Vo = R0, V0
        del R0, V0
        for s in range(n_steps):
            Ro, Vo, mom = oracle.run(Ro, Vo, w, dt, eps, K, 1, oracle.FIELD_POISSON, nr=nr,
                                     rmin=-RMAX, rmax=RMAX, with_moments=True)
            sim.step(dt, eps, EP_FIELD_POISSON, 1)
            parts = [sim.particles(a, c) for a, c in ranges]
            R = np.concatenate([p[0] for p in parts])
            V = np.concatenate([p[1] for p in parts])
            err = rel_particle(R, V, Ro[idx], Vo[idx], BEAM_SIZE)
            worst = max(worst, float(err.max()))
            assert err.max() <= TOL_PARTICLE, (s, err.max())
            m = sim.moments(eps, EP_FIELD_POISSON)
            mo = dict(zip(oracle.MOMENT_NAMES, mom[-1]))
            for k in ("rms_radius", "energy"):
                assert abs(m[k] - mo[k]) <= TOL_RUN * abs(mo[k]), (s, k, m[k], mo[k])
            assert m["n_nan"] == 0 and m["n_offmesh"] == mo["n_offmesh"]
    return worst


def test_full_size_parity_vp_1e6():
    """N_p = 1e6, N_r = 256, eps = 0.01, dt = 0.05."""
    full_size_parity(1_000_000, 256, 0.01, 0.05, 4, 5, 20000, seed=12)


def test_full_size_parity_vp_8e6_substeps():
    """N_p = 8e6 (long enough for the push's two-group form and its gather
    without range tests), N_r = 4096, eps = 1e-3, dt = 0.05, K = 16, with
    particles around the mesh edge in the first wave."""
    full_size_parity(8_000_000, 4096, 1e-3, 0.05, 16, 3, 20000, seed=14, edge=True)


def test_full_size_parity_vp_1e8():
    """N_p = 1e8, N_r = 4096, eps = 1e-3, dt = 0.05, K = 1 (the benchmark shape)."""
    full_size_parity(100_000_000, 4096, 1e-3, 0.05, 1, 3, 20000, seed=13)


def test_full_size_parity_vp_1e8_eps_1e2():
    """The benchmark shape at the configuration's other eps: N_p = 1e8,
    N_r = 4096, eps = 1e-2, dt = 0.05, K = 1."""
    full_size_parity(100_000_000, 4096, 1e-2, 0.05, 1, 3, 20000, seed=13)


def test_statistical_rms_1e8_against_oracle_subsample():
    """Full physics at scale, pinned statistically: the GPU run at N_p = 1e8
    (N_r = 4096, eps = 1e-3, dt = 0.05, K = 1) against the oracle's own
    self-consistent run of the beam's first 1e6 particles (weight 1e-6).  The
    rms radii agree within 3/sqrt(N_sub) at every recorded step, the sampling
    noise of the sub-beam."""
    n, n_sub, steps, every, nr, eps, dt = 100_000_000, 1_000_000, 40, 10, 4096, 1e-3, 0.05
    R0, V0, w = synth.gaussian_truncated(n, seed=13)
    Rs, Vs = R0[:n_sub].copy(), V0[:n_sub].copy()
    gpu = []
    with Sim(n, n_cells=nr, substeps=1) as sim:
        sim.set_particles(R0, V0, w)
        del R0, V0
        gpu.append(sim.moments(eps, EP_FIELD_POISSON)["rms_radius"])
        for _ in range(steps // every):
            sim.step(dt, eps, EP_FIELD_POISSON, every)
            gpu.append(sim.moments(eps, EP_FIELD_POISSON)["rms_radius"])
    _, _, mom = oracle.run(Rs, Vs, 1.0 / n_sub, dt, eps, 1, steps, oracle.FIELD_POISSON, nr=nr,
                           rmin=-RMAX, rmax=RMAX, with_moments=True)
    orc = mom[::every, 1]
    rel = np.abs(np.array(gpu) - orc) / orc
    assert rel.max() <= 3.0 / math.sqrt(n_sub), rel


@pytest.mark.timeout(900)
@pytest.mark.parametrize("eps", [1e-3, 1e-2])
def test_statistical_rms_1e8_full_run(eps):
    """The at-scale configuration over its full length: 1e4 steps of the
    1e8-particle beam (N_r = 4096, dt = 0.05, K = 1) on the GPU against the
    oracle's own self-consistent run of the beam's first 1e6 particles
    (weight 1e-6) over the same 1e4 steps.  The rms radii agree within
    3/sqrt(N_sub), the sub-beam's sampling noise, every 500 steps."""
    n, n_sub, steps, every, nr, dt = 100_000_000, 1_000_000, 10_000, 500, 4096, 0.05
    R0, V0, w = synth.gaussian_truncated(n, seed=13)
    Rs, Vs = R0[:n_sub].copy(), V0[:n_sub].copy()
    gpu = []
    with Sim(n, n_cells=nr, substeps=1) as sim:
        sim.set_particles(R0, V0, w)
        del R0, V0
        gpu.append(sim.moments(eps, EP_FIELD_POISSON)["rms_radius"])
        for _ in range(steps // every):
            sim.step(dt, eps, EP_FIELD_POISSON, every)
            m = sim.moments(eps, EP_FIELD_POISSON)
            gpu.append(m["rms_radius"])
        assert m["n_nan"] == 0 and m["n_steps"] == steps
    print("gpu run done eps=%g, oracle sub-beam of %d for %d steps" % (eps, n_sub, steps),
          flush=True)
    _, _, mom = oracle.run(Rs, Vs, 1.0 / n_sub, dt, eps, 1, steps, oracle.FIELD_POISSON, nr=nr,
                           rmin=-RMAX, rmax=RMAX, with_moments=True)
    orc = mom[::every, 1]
    rel = np.abs(np.array(gpu) - orc) / orc
    assert rel.max() <= 3.0 / math.sqrt(n_sub), rel
