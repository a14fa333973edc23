"""Period and modulus diagnostics of the paper (section 2 and section 4):
each particle's period and its ratio to 2 pi eps, the spread of the periods,
how they and the modulus |(R, V)| change along a run.  The periods come from
the library's fine-solve search (ep_compute_periods), the states from
ep_get_particles; the summaries below are host reductions of those arrays.
"""
import math

import numpy as np

from . import capi


def period_summary(sim, eps, field, bins=32):
    """Periods of the context's current state: mean, spread, their ratio to
    2 pi eps, a histogram and the per-particle array."""
    un = capi.ep_compute_periods(sim.ctx, eps, field)
    T, _, _ = capi.ep_get_periods(sim.ctx, sim.n)
    free = 2.0 * math.pi * eps
    hist, edges = np.histogram(T / free, bins=bins)
    return {"mean": float(T.mean()), "std": float(T.std()), "min": float(T.min()),
            "max": float(T.max()), "mean_over_2pi_eps": float(T.mean() / free),
            "unresolved": un, "histogram": hist.tolist(),
            "bin_edges_over_2pi_eps": edges.tolist()}, T


def modulus_change(R0, V0, R, V):
    """|y(t)| against |y(0)| per particle: mean and spread of the ratio, the
    largest relative change."""
    a0 = np.hypot(R0, V0)
    a = np.hypot(R, V)
    ok = a0 > 0
    r = a[ok] / a0[ok]
    return {"ratio_mean": float(r.mean()), "ratio_std": float(r.std()),
            "max_relative_change": float(np.max(np.abs(r - 1.0)))}


def period_change(T0, T):
    """Periods at a later time against the initial ones."""
    r = T / T0
    return {"ratio_mean": float(r.mean()), "ratio_std": float(r.std()),
            "correlation": float(np.corrcoef(T0, T)[0, 1])}
