"""Seeded synthetic particle beams shared by the tests, the benchmark and the
smoke check.

Draws only: no step of the method lives here.  Every generator uses numpy's
``default_rng(seed)`` and returns FP64 arrays (R, V) and the uniform weight.
The draws are rounded to FP32-representable values, so that a consumer which
stores particles in FP32 and one which computes in FP64 start from exactly the
same numbers.

Workloads (the paper's experiments draw macroparticles from the density of
f0, section 2.1; the configurations below are synthetic beams of that kind):
  * ``gaussian_truncated``: R ~ N(0, sigma) truncated to |R| < cut by
    rejection, V ~ N(0, sigma); the Vlasov-Poisson beams.
  * ``gaussian``: R, V ~ N(0, sigma) i.i.d.; the Duffing beams.
  * ``paper_f0``: eq. (2.7) of the paper: R uniform on [-0.75, 0.75],
    V ~ N(0, v_th) with v_th = 0.0727518214392.
"""
import numpy as np

V_TH_PAPER = 0.0727518214392


def _fp32(a):
    return a.astype(np.float32).astype(np.float64)


def gaussian(n, seed, sigma=1.0):
    rng = np.random.default_rng(seed)
    R = rng.standard_normal(n) * sigma
    V = rng.standard_normal(n) * sigma
    return _fp32(R), _fp32(V), 1.0 / max(n, 1)


def gaussian_truncated(n, seed, sigma=1.0, cut=4.0):
    rng = np.random.default_rng(seed)
    R = np.empty(n)
    filled = 0
    while filled < n:
        draw = rng.standard_normal(max(1024, int((n - filled) * 1.01))) * sigma
        draw = draw[np.abs(draw) < cut][: n - filled]
        R[filled:filled + draw.size] = draw
        filled += draw.size
    V = rng.standard_normal(n) * sigma
    return _fp32(R), _fp32(V), 1.0 / max(n, 1)


def paper_f0(n, seed, v_th=V_TH_PAPER, half_width=0.75):
    rng = np.random.default_rng(seed)
    R = rng.uniform(-half_width, half_width, n)
    V = rng.standard_normal(n) * v_th
    return _fp32(R), _fp32(V), 1.0 / max(n, 1)


def nodes_exact(nr, rmax):
    """Mesh node coordinates x_k = -rmax + k*hr (exact for power-of-two nr
    and rmax = 5 up to one rounding of k*hr)."""
    hr = 2.0 * rmax / nr
    return -rmax + np.arange(nr + 1) * hr


def mlp_init(n_in, hidden, n_out, seed):
    """Random-init weights of the corrector MLP (Glorot-uniform, zero biases),
    FP32, packed as W1[hidden,n_in], b1, W2[hidden,hidden], b2, W3[n_out,hidden], b3."""
    rng = np.random.default_rng(seed)

    def glorot(fan_out, fan_in):
        a = np.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-a, a, (fan_out, fan_in))

    parts = [glorot(hidden, n_in), np.zeros(hidden), glorot(hidden, hidden), np.zeros(hidden),
             glorot(n_out, hidden), np.zeros(n_out)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)
