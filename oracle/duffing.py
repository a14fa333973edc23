"""Exact Duffing characteristics and periods (appendix A of the paper).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

With E = -R^3 the characteristics (eq. 1.4) reduce to the undamped Duffing
equation R'' + R/eps^2 + R^3/eps = 0, R(0) = r0, R'(0) = v0/eps (eq. 1.5 / A.1).
Its orbits are level sets of the energy; the paper writes the Hamiltonian with
R' as momentum; in the (R, V = eps R') variables of eq. 1.4 the conserved
quantity is eps times it:  H(R, V) = (R^2 + V^2)/(2 eps) + R^4/4.

The solution is a Jacobi elliptic cosine (appendix A, first paragraph):
  R(t) = b cn(w t + u0 | m),    V(t) = eps R'(t) = -eps b w sn dn,
  w^2 = 1/eps^2 + b^2/eps,      m = eps b^2 / (2 (1 + eps b^2)),
with the turning point b of eq. (A.5) and u0 fixed by the initial data.
The exact period is T = 4 K(m) / w; eqs. (A.7)/(A.8) give its expansions.
"""
import numpy as np
from scipy import special


def turning_point(r0, v0, eps):
    """b of eq. (A.5): the positive R where the orbit crosses V = 0."""
    r0 = np.asarray(r0, dtype=np.float64)
    v0 = np.asarray(v0, dtype=np.float64)
    return np.sqrt((np.sqrt(1.0 + 2.0 * eps * (r0 ** 2 + v0 ** 2) + eps ** 2 * r0 ** 4) - 1.0)
                   / eps)


def energy(R, V, eps):
    """Conserved energy of eq. 1.4 with E = -R^3 (eps times the paper's H)."""
    R = np.asarray(R, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    return (R ** 2 + V ** 2) / (2.0 * eps) + R ** 4 / 4.0


def _params(r0, v0, eps):
    b = turning_point(r0, v0, eps)
    w = np.sqrt(1.0 / eps ** 2 + b ** 2 / eps)
    m = eps * b ** 2 / (2.0 * (1.0 + eps * b ** 2))
    return b, w, m


def period(r0, v0, eps):
    """Exact period T = 4 K(m) / w."""
    b, w, m = _params(r0, v0, eps)
    return 4.0 * special.ellipk(m) / w


def period_series_b(r0, v0, eps):
    """Eq. (A.7): T = 2 pi eps - (3 pi/4) b^2 eps^2 + (57 pi/128) b^4 eps^3."""
    b = turning_point(r0, v0, eps)
    return 2 * np.pi * eps - 0.75 * np.pi * b ** 2 * eps ** 2 + 57.0 * np.pi / 128.0 * b ** 4 * eps ** 3


def period_series_initial(r0, v0, eps):
    """Eq. (A.8): the expansion in the initial data."""
    r0 = np.asarray(r0, dtype=np.float64)
    v0 = np.asarray(v0, dtype=np.float64)
    a2 = r0 ** 2 + v0 ** 2
    return (2 * np.pi * eps - 0.75 * np.pi * a2 * eps ** 2
            + (105.0 * np.pi / 128.0 * a2 ** 2 - 3.0 * np.pi / 8.0 * r0 ** 4) * eps ** 3)


def solution(r0, v0, eps, t):
    """Exact (R(t), V(t)) of the Duffing characteristics from (r0, v0) at time t."""
    r0 = np.asarray(r0, dtype=np.float64)
    v0 = np.asarray(v0, dtype=np.float64)
    b, w, m = _params(r0, v0, eps)
    safe_b = np.where(b > 0, b, 1.0)
    phi = np.arccos(np.clip(r0 / safe_b, -1.0, 1.0))
    # V(0) = -eps b w sn(u0) dn(u0) = v0: u0 < 0 when v0 > 0, u0 >= 0 otherwise
    # (v0 = 0 and r0 = -b gives u0 = F(pi | m) = 2 K(m), where cn = -1)
    u0 = np.where(v0 > 0, -1.0, 1.0) * special.ellipkinc(phi, m)
    sn, cn, dn, _ = special.ellipj(w * t + u0, m)
    R = b * cn
    V = -eps * b * w * sn * dn
    return R, V
