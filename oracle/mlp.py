"""FP64 oracle of the learned Duhamel corrector (network, training step and
learned push).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Plain numpy in FP64;
``@`` (matmul) is the only library primitive used for the layers.

Network (5 or 6 inputs -> 64 -> 64 -> 2):
    h1 = act(W1 x + b1),  h2 = act(W2 h1 + b2),  o = W3 h2 + b3
with the inverse-square-root unit act(z) = z / sqrt(1 + z^2) (Carlile et al.,
2017), a smooth odd saturating activation like tanh; act'(z) = (1 + z^2)^(-3/2).
Parameters are one flat FP32/FP64 vector in the order W1[64,n_in], b1[64],
W2[64,64], b2[64], W3[2,64], b3[2] (row-major).

Features of a particle y_n = (R, V) for a step dt at eps:
    x = (R / s_in, V / s_in, cos phi, sin phi, (dt/eps) / s_t [, E^n(R) / s_E])
with phi = (dt/eps) mod 2 pi.

Output map.  The exact step is y_{n+1} = r(dt/eps) y_n + D (eq. 3.6, D the
Duhamel term).  The network gives D in polar form around the exact rotation:
    delta = mu_d + sig_d o_0  (phase advance beyond dt/eps)
    kappa = mu_k + sig_k o_1  (relative change of |y|)
    y_{n+1} = (1 + kappa) r(dt/eps + delta) y_n,   D = y_{n+1} - r(dt/eps) y_n
or, with the amplitude-scaled map (out_map = 1), the arc length and the
radial displacement of the step beyond the free rotation,
    s = mu_d + sig_d o_0 = a delta,   rho = mu_k + sig_k o_1 = a kappa,
    a = |y_n|, i.e. delta = s / a and kappa = rho / a.
In the self-consistent field E(0+) = rho(0) > 0 = -E(0-), so the phase
advance of small orbits grows like 1/a while s and rho stay bounded: the
scaled targets are the ones a smooth network can fit there.

Base push (base_K > 0, Duffing field).  The same polar map can act around
the plain K_b-substep step y_b of y_n instead of the free rotation:
    y_{n+1} = (1 + kappa) r(delta) y_b,
so that (delta, kappa) is the plain push's defect against the fine push, a
correction that shrinks like K_b^-2 where the plain push converges at second
order; with base_K = 0, y_b = r(dt/eps) y_n and the two forms agree.
Check: the frozen-field energy H^n(y) = (R^2 + V^2)/(2 eps) + P(R), P = R^4/4
(Duffing) or the mesh potential Psi^n (Poisson), must satisfy
|H^n(y_{n+1}) - H^n(y_n)| <= tol |H^n(y_n)|; particles that fail take the
plain K_fb-substep push instead.  Projection (optional): the exact step
conserves H^n (the Duffing energy, or the frozen-field energy of the step),
so every particle of the step (the network's and the fallback's) may be
moved radially back onto its energy shell with one Newton step
(project_energy); the phase of the result is kept.

Parity unpinned: nothing (forward/backward pinned by finite differences and
the linear limit, Adam by its closed-form first step, the output map by the
exact free rotation and the label round trip).
"""
import math

import numpy as np

HIDDEN = 64
N_OUT = 2


def n_params(n_in):
    return HIDDEN * n_in + HIDDEN + HIDDEN * HIDDEN + HIDDEN + N_OUT * HIDDEN + N_OUT


def unpack(p, n_in):
    p = np.asarray(p, dtype=np.float64)
    assert p.size == n_params(n_in)
    shapes = [(HIDDEN, n_in), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (N_OUT, HIDDEN), (N_OUT,)]
    out, o = [], 0
    for s in shapes:
        k = int(np.prod(s))
        out.append(p[o:o + k].reshape(s))
        o += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in parts])


def act(z):
    return z / np.sqrt(1.0 + z * z)


def act_grad(z):
    return (1.0 + z * z) ** -1.5


def forward(p, X, n_in=None):
    """X: [B, n_in].  Returns (O [B, 2], cache)."""
    X = np.asarray(X, dtype=np.float64)
    n_in = X.shape[1] if n_in is None else n_in
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in)
    z1 = X @ W1.T + b1
    h1 = act(z1)
    z2 = h1 @ W2.T + b2
    h2 = act(z2)
    O = h2 @ W3.T + b3
    return O, (X, z1, h1, z2, h2, W1, W2, W3)


def backward(cache, dO):
    """Gradient of sum(dO * O) with respect to the flat parameter vector."""
    X, z1, h1, z2, h2, W1, W2, W3 = cache
    dO = np.asarray(dO, dtype=np.float64)
    dW3 = dO.T @ h2
    db3 = dO.sum(0)
    dz2 = (dO @ W3) * act_grad(z2)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * act_grad(z1)
    dW1 = dz1.T @ X
    db1 = dz1.sum(0)
    return pack([dW1, db1, dW2, db2, dW3, db3])


def mse_loss_grad(p, X, Y):
    """Loss = mean over the batch and the two outputs of (O - Y)^2."""
    O, cache = forward(p, X)
    B = X.shape[0]
    diff = O - np.asarray(Y, dtype=np.float64)
    loss = float(np.mean(diff * diff))
    dO = 2.0 * diff / (B * N_OUT)
    return loss, backward(cache, dO)


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) at step t >= 1; returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------ model

class Norm:
    """Normalisation constants of a trained corrector (stored with its weights)."""

    def __init__(self, s_in=1.5, s_t=100.0, s_E=1.0, mu_d=0.0, sig_d=1.0, mu_k=0.0, sig_k=1.0,
                 out_map=0, base_K=0):
        self.s_in, self.s_t, self.s_E = s_in, s_t, s_E
        self.mu_d, self.sig_d, self.mu_k, self.sig_k = mu_d, sig_d, mu_k, sig_k
        self.out_map = int(out_map)   # 0: (delta, kappa); 1: (a delta, a kappa)
        self.base_K = int(base_K)     # 0: around the free rotation; K: around the plain K push

    def as_array(self):
        return np.array([self.s_in, self.s_t, self.s_E, self.mu_d, self.sig_d, self.mu_k,
                         self.sig_k, float(self.out_map), float(self.base_K)])

    @classmethod
    def from_array(cls, a):
        return cls(*[float(x) for x in a[:7]], out_map=int(a[7]),
                   base_K=int(a[8]) if len(a) > 8 else 0)


def features(R, V, dt, eps, norm, Egather=None):
    th = dt / eps
    phi = math.fmod(th, 2.0 * math.pi)
    cols = [R / norm.s_in, V / norm.s_in, np.full_like(R, math.cos(phi)),
            np.full_like(R, math.sin(phi)), np.full_like(R, th / norm.s_t)]
    if Egather is not None:
        cols.append(Egather / norm.s_E)
    return np.stack(cols, axis=1)


def rotate(phi, R, V):
    """y <- r(phi) y, r of eq. 3.3 with T = 2 pi (phi may be an array)."""
    c, s = np.cos(phi), np.sin(phi)
    return c * R + s * V, -s * R + c * V


def apply_polar(R, V, dt, eps, delta, kappa, scaled=False):
    """y_{n+1} = (1 + kappa) r(dt/eps + delta) y_n; with scaled=True the
    inputs are (a delta, a kappa), a = |y_n| (nothing moves at a = 0)."""
    if scaled:
        a = np.hypot(R, V)
        inv = np.divide(1.0, a, out=np.zeros_like(a), where=a > 0)
        delta, kappa = delta * inv, kappa * inv
    R1, V1 = rotate(dt / eps + delta, R, V)
    return (1.0 + kappa) * R1, (1.0 + kappa) * V1


def polar_labels(R, V, R1, V1, dt, eps, scaled=False):
    """Inverse of apply_polar: (delta, kappa) that map y_n to y_{n+1}.
    delta is the angle from r(dt/eps) y_n to y_{n+1} in the direction in which
    r advances (atan2 of the cross and dot products), kappa = |y_{n+1}|/|y_n| - 1;
    scaled=True returns (a delta, |y_{n+1}| - a), a = |y_n|."""
    uR, uV = rotate(dt / eps, R, V)
    delta = np.arctan2(R1 * uV - V1 * uR, R1 * uR + V1 * uV)
    a = np.hypot(R, V)
    if scaled:
        return a * delta, np.hypot(R1, V1) - a
    kappa = np.hypot(R1, V1) / a - 1.0
    return delta, kappa


def apply_polar_to(Rb, Vb, delta, kappa, scaled=False):
    """y_{n+1} = (1 + kappa) r(delta) y_b around a base point y_b (the base
    push's result); scaled=True takes (a delta, a kappa) with a = |y_b|."""
    if scaled:
        a = np.hypot(Rb, Vb)
        inv = np.divide(1.0, a, out=np.zeros_like(a), where=a > 0)
        delta, kappa = delta * inv, kappa * inv
    R1, V1 = rotate(delta, Rb, Vb)
    return (1.0 + kappa) * R1, (1.0 + kappa) * V1


def polar_labels_from(Rb, Vb, R1, V1, scaled=False):
    """Inverse of apply_polar_to: delta = angle from y_b to y_{n+1} in the
    direction in which r advances, kappa = |y_{n+1}|/|y_b| - 1 (scaled:
    (a delta, |y_{n+1}| - a), a = |y_b|)."""
    delta = np.arctan2(R1 * Vb - V1 * Rb, R1 * Rb + V1 * Vb)
    a = np.hypot(Rb, Vb)
    if scaled:
        return a * delta, np.hypot(R1, V1) - a
    return delta, np.hypot(R1, V1) / a - 1.0


def predict(p, R, V, dt, eps, norm, Egather=None):
    """Network prediction for particles (R, V): (delta, kappa), or (a delta,
    a kappa) with the amplitude-scaled map."""
    X = features(R, V, dt, eps, norm, Egather)
    O, _ = forward(p, X)
    return norm.mu_d + norm.sig_d * O[:, 0], norm.mu_k + norm.sig_k * O[:, 1]


def energy(R, V, eps, potential):
    return (R * R + V * V) / (2.0 * eps) + potential(R)


def project_energy(R1, V1, H0, eps, potential, dpotential):
    """One Newton step of the radial projection y <- s y onto the energy shell
    H(y) = H0 (H = |y|^2/(2 eps) + P(R)) from s = 1:
    s = 1 - (H(y) - H0) / (dH(s y)/ds at s = 1), with
    dH/ds = |y|^2 / eps + R P'(R).  From a point within tol of the shell the
    projected energy is off by O(tol^2).  Where the slope is not above half
    of its kinetic part |y|^2 / eps (small orbits in a field that points
    outward) the point is left as it is."""
    A = (R1 * R1 + V1 * V1) / eps
    slope = A + R1 * dpotential(R1)
    ok = slope > 0.5 * A
    s = 1.0 - (energy(R1, V1, eps, potential) - H0) / np.where(ok, slope, 1.0)
    s = np.where(ok, s, 1.0)
    return s * R1, s * V1


def learned_step(p, R, V, dt, eps, norm, potential, plain_push, tol, Egather=None,
                 base_push=None, dpotential=None):
    """One learned step with energy check and plain fallback.

    potential(R): the frozen-field potential P of H^n; plain_push(R, V): the
    plain step used for particles that fail the check; base_push(R, V): the
    plain step with norm.base_K substeps, which a network with a base push
    corrects (needed then, unused otherwise); dpotential(R) = P'(R): given,
    every particle, the network's and the fallback's, is projected onto its
    energy shell H^n(y_{n+1}) = H^n(y_n) (project_energy) after the check.
    Returns (R1, V1, fell_back[bool], ratio = |dH|/|H| of the network's
    prediction, before the projection)."""
    delta, kappa = predict(p, R, V, dt, eps, norm, Egather)
    if norm.base_K:
        if base_push is None:
            raise ValueError("the network corrects the plain push with %d substeps: "
                             "pass base_push" % norm.base_K)
        Rb, Vb = base_push(R, V)
        R1, V1 = apply_polar_to(Rb, Vb, delta, kappa, scaled=norm.out_map == 1)
    else:
        R1, V1 = apply_polar(R, V, dt, eps, delta, kappa, scaled=norm.out_map == 1)
    H0 = energy(R, V, eps, potential)
    H1 = energy(R1, V1, eps, potential)
    ratio = np.abs(H1 - H0) / np.abs(H0)
    fb = ~(ratio <= tol)
    if np.any(fb):
        Rf, Vf = plain_push(R[fb], V[fb])
        R1 = R1.copy()
        V1 = V1.copy()
        R1[fb] = Rf
        V1[fb] = Vf
    if dpotential is not None:
        R1, V1 = project_energy(R1, V1, H0, eps, potential, dpotential)
    return R1, V1, fb, ratio
