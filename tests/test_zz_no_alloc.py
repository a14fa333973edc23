"""The no-allocation step (ep_step_noalloc) against the context path.

ep_step_noalloc runs ep_step's kernels on caller-owned FP32 device arrays with
its working memory in a static device array.  Each case steps the same beam
once through a context (ep_bind_particles on one pair of caller arrays,
ep_step) and once through ep_step_noalloc (another pair), twice in a row on
the same device -- the second call with a smaller beam, so it runs on the
static memory the first left behind -- and compares the rotating-frame states
bitwise (integer fixed-point deposit and the same launches: the bar of the
plain path's own determinism tests) and the returned phase with the
context's."""
import numpy as np
import pytest

from paper_1404_1160_amd import (EP_FIELD_DUFFING, EP_FIELD_POISSON, EP_FIELD_ZERO, Sim, capi,
                                 synth)
from test_gpu_boundary import Hip

pytestmark = pytest.mark.gpu


def _context_run(hip, R0, V0, w, field, nr, K, dt, eps, steps):
    n = R0.size
    dR, dV = hip.malloc(4 * n), hip.malloc(4 * n)
    try:
        hip.upload(dR, R0.astype(np.float32))
        hip.upload(dV, V0.astype(np.float32))
        with Sim(n, n_cells=nr, substeps=K) as sim:
            capi.ep_bind_particles(sim.ctx, dR, dV, n, w)
            for k in steps:
                sim.step(dt, eps, field, k)
            phase = sim.moments(eps, field)["phase"]
        return hip.download(dR, n, np.float32), hip.download(dV, n, np.float32), phase
    finally:
        hip.free(dR)
        hip.free(dV)


def _noalloc_run(hip, R0, V0, w, field, nr, K, dt, eps, steps, stream=None):
    n = R0.size
    dR, dV = hip.malloc(4 * n), hip.malloc(4 * n)
    try:
        hip.upload(dR, R0.astype(np.float32))
        hip.upload(dV, V0.astype(np.float32))
        phase = 0.0
        for k in steps:
            phase = capi.ep_step_noalloc(dR, dV, n, w, dt, eps, field, k, phase, n_cells=nr,
                                         r_max=5.0, substeps=K, hip_stream=stream)
        if stream is not None:
            hip.stream_sync(stream)
        return hip.download(dR, n, np.float32), hip.download(dV, n, np.float32), phase
    finally:
        hip.free(dR)
        hip.free(dV)


CASES = [
    # field, N_r, K, dt, eps, steps per call (a list: consecutive calls)
    (EP_FIELD_POISSON, 4096, 1, 0.05, 1e-3, [3, 4]),
    (EP_FIELD_POISSON, 256, 64, 0.05, 0.01, [600]),     # 38400 coefficients: two table fills
    (EP_FIELD_DUFFING, 256, 8, 0.1, 0.05, [5, 1]),
]


@pytest.mark.parametrize("field,nr,K,dt,eps,steps", CASES)
def test_noalloc_step_equals_context_step(field, nr, K, dt, eps, steps):
    hip = Hip()
    st = hip.stream()
    try:
        for n, seed in ((1_000_003, 71), (10_001, 72)):
            R0, V0, w = synth.gaussian_truncated(n, seed=seed)
            if len(steps) == 1 and steps[0] * K > 2 ** 15 and n > 100_000:
                continue     # the long case runs on the small beam only
            a = _context_run(hip, R0, V0, w, field, nr, K, dt, eps, steps)
            b = _noalloc_run(hip, R0, V0, w, field, nr, K, dt, eps, steps, stream=st)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), (n, field)
            assert np.all(np.isfinite(b[0])) and not np.array_equal(b[0], R0.astype(np.float32))
            assert a[2] == b[2], (a[2], b[2])
    finally:
        hip.stream_destroy(st)


def test_noalloc_free_rotation_and_limits():
    hip = Hip()
    d = hip.malloc(4 * 64)
    try:
        # E = 0 only advances the phase; the state is left as it is
        hip.upload(d, np.arange(32, dtype=np.float32))
        ph = capi.ep_step_noalloc(d, d + 128, 32, 1.0, 0.1, 0.05, EP_FIELD_ZERO, 7, 0.5)
        assert ph == pytest.approx(np.fmod(0.5 + 7 * np.fmod(2.0, 2 * np.pi), 2 * np.pi), abs=1e-12)
        assert np.array_equal(hip.download(d, 32, np.float32), np.arange(32, dtype=np.float32))
        bad = [dict(n_cells=16384), dict(n_cells=255), dict(substeps=2 ** 15 + 1),
               dict(substeps=0)]
        for kw in bad:
            args = dict(n_cells=256, r_max=5.0, substeps=1)
            args.update(kw)
            with pytest.raises(capi.EtdpicError) as e:
                capi.ep_step_noalloc(d, d + 128, 32, 1.0, 0.05, 0.01, EP_FIELD_POISSON, 1, 0.0,
                                     **args)
            assert e.value.status == capi.EP_EINVAL
            assert "ep_step_noalloc" in capi.ep_last_error(None)
        with pytest.raises(capi.EtdpicError) as e:
            capi.ep_step_noalloc(d + 4, d + 128, 32, 1.0, 0.05, 0.01, EP_FIELD_POISSON, 1, 0.0)
        assert e.value.status == capi.EP_EINVAL
    finally:
        hip.free(d)
