"""Checkpoint and resume (ep_save / ep_load) through the C ABI.

A run interrupted by a save, a fresh context and a load must continue bit for
bit: the particles are stored in FP32 as held, the phase and clock in FP64,
and the field is recomputed from the restored particles with the same
fixed-point deposit.
"""
import numpy as np
import pytest

from oracle import mlp
from paper_1404_1160_amd import (EP_DEPOSIT_ATOMIC, EP_DEPOSIT_SORTED, EP_FIELD_DUFFING,
                                 EP_FIELD_POISSON, EP_MLP_BF16, EP_MLP_FP16, EP_PUSH_IMPROVED_ETD,
                                 EP_PUSH_LEARNED, EtdpicError, Sim, capi, synth)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("deposit", [EP_DEPOSIT_ATOMIC, EP_DEPOSIT_SORTED])
def test_poisson_resume_is_bitwise(tmp_path, deposit):
    R, V, w = synth.paper_f0(300_007, seed=31)
    dt, eps = 0.05, 1e-2
    kw = dict(n_cells=512, substeps=2, deposit=deposit)
    path = str(tmp_path / "ck.bin")
    with Sim(R.size, **kw) as a:
        a.set_particles(R, V, w)
        a.step(dt, eps, EP_FIELD_POISSON, 7)
        a.save(path)
        a.step(dt, eps, EP_FIELD_POISSON, 9)
        Ra, Va = a.particles()
        ma = a.moments(eps, EP_FIELD_POISSON)
    with Sim(R.size + 100, **kw) as b:
        b.load(path)
        assert b.n == R.size
        b.step(dt, eps, EP_FIELD_POISSON, 9)
        Rb, Vb = b.particles()
        mb = b.moments(eps, EP_FIELD_POISSON)
    assert np.array_equal(Ra, Rb) and np.array_equal(Va, Vb)
    for k in ("t", "phase", "charge", "n_steps", "n_offmesh"):
        assert ma[k] == mb[k], k
    # The sorted context holds the particles in cell order, the restored one
    # in loaded order until its next sort, so the FP64 moment sums run in a
    # different order: equal to rounding then, bitwise for the atomic deposit.
    rtol = 0.0 if deposit == EP_DEPOSIT_ATOMIC else 1e-13
    for k in ("rms_radius", "energy", "kinetic", "potential"):
        assert abs(ma[k] - mb[k]) <= rtol * abs(ma[k]), k


@pytest.mark.parametrize("precision", [EP_MLP_BF16, EP_MLP_FP16])
def test_learned_resume_restores_network(tmp_path, precision):
    """The network, its normalisation, the push mode and the inference
    precision come back: the resumed run matches bit for bit (the two
    precisions give different bits, so a lost setting would show)."""
    R, V, w = synth.gaussian(50_001, seed=32, sigma=1.5)
    dt, eps = 0.05, 1e-3
    p = synth.mlp_init(5, 64, 2, seed=3)
    norm = np.array([1.5, 100.0, 1.0, 0.0, 0.01, 0.0, 1e-3, 0.0, 0.0])
    path = str(tmp_path / "ck.bin")
    with Sim(R.size, substeps=16) as a:
        capi.ep_mlp_set_weights(a.ctx, p, norm)
        capi.ep_set_push_mode(a.ctx, EP_PUSH_LEARNED, 1e-4, 32)
        capi.ep_mlp_set_precision(a.ctx, precision)
        a.set_particles(R, V, w)
        a.step(dt, eps, EP_FIELD_DUFFING, 3)
        a.save(path)
        a.step(dt, eps, EP_FIELD_DUFFING, 4)
        Ra, Va = a.particles()
    with Sim(R.size, substeps=16) as b:
        capi.ep_mlp_set_precision(b.ctx, EP_MLP_FP16 + EP_MLP_BF16 - precision)
        b.load(path)
        q, nb = capi.ep_mlp_get_weights(b.ctx, mlp.n_params(5))
        assert np.array_equal(q, p.astype(np.float32))
        assert np.array_equal(nb, norm)
        b.step(dt, eps, EP_FIELD_DUFFING, 4)
        Rb, Vb = b.particles()
    assert np.array_equal(Ra, Rb) and np.array_equal(Va, Vb)


def test_fine_solver_resume_restores_mode_and_step(tmp_path):
    """The improved ETD push mode and the fine step h_fine come back with the
    checkpoint: the resumed run matches bit for bit."""
    R, V, w = synth.paper_f0(2_001, seed=34)
    dt, eps, h = 0.2, 1e-2, 2.0 * np.pi * 1e-2 / 50
    path = str(tmp_path / "ck.bin")
    with Sim(R.size, substeps=4) as a:
        capi.ep_set_push_mode(a.ctx, EP_PUSH_IMPROVED_ETD)
        capi.ep_set_fine_solver(a.ctx, h, 5000)
        a.set_particles(R, V, w)
        a.step(dt, eps, EP_FIELD_DUFFING, 2)
        a.save(path)
        a.step(dt, eps, EP_FIELD_DUFFING, 2)
        Ra, Va = a.particles()
        Ta, Na, _ = capi.ep_get_periods(a.ctx, R.size)
    with Sim(R.size, substeps=4) as b:
        b.load(path)
        # the kept periods come back too: the resumed steps reuse them
        Tl, _, _ = capi.ep_get_periods(b.ctx, R.size)
        b.step(dt, eps, EP_FIELD_DUFFING, 2)
        Rb, Vb = b.particles()
        Tb, Nb, _ = capi.ep_get_periods(b.ctx, R.size)
    assert np.array_equal(Ra, Rb) and np.array_equal(Va, Vb)
    assert np.array_equal(Tl, Ta) and np.array_equal(Tb, Ta) and np.array_equal(Nb, Na)


def test_load_rejects_mismatch_and_garbage(tmp_path):
    R, V, w = synth.gaussian(1000, seed=33)
    path = str(tmp_path / "ck.bin")
    with Sim(R.size, n_cells=256) as a:
        a.set_particles(R, V, w)
        a.save(path)
    with Sim(R.size, n_cells=128) as b:
        with pytest.raises(EtdpicError) as e:
            b.load(path)
        assert e.value.status == capi.EP_EINVAL
    with Sim(R.size - 1, n_cells=256) as b:
        with pytest.raises(EtdpicError) as e:
            b.load(path)
        assert e.value.status == capi.EP_EINVAL
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"not a checkpoint at all" * 10)
    with Sim(R.size) as b:
        with pytest.raises(EtdpicError) as e:
            b.load(str(bad))
        assert e.value.status == capi.EP_EIO
        with pytest.raises(EtdpicError) as e:
            b.load(str(tmp_path / "missing.bin"))
        assert e.value.status == capi.EP_EIO
    data = open(path, "rb").read()
    (tmp_path / "short.bin").write_bytes(data[: len(data) // 2])
    with Sim(R.size) as b:
        with pytest.raises(EtdpicError) as e:
            b.load(str(tmp_path / "short.bin"))
        assert e.value.status == capi.EP_EIO
