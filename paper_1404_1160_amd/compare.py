"""Equal-error comparison of the plain push and the learned corrector.

Duffing workload (`equal_error`): eps = 1e-3, dt = 0.05,
R, V ~ N(0, 1.5); the network (5 -> 64 -> 64 -> 2) is trained on the GPU on
samples labelled by the plain push with K_fine substeps, then both forms push
an evaluation beam for `steps` steps.  Error = the largest relative
rms-radius error over the run (recorded every `every` steps) against a
reference run of the plain push with K_ref substeps; the maximum over the run
rather than the final value, because the signed final error of a single run
can pass through zero by chance.  Throughput = particle-steps/s of the whole
run (wall clock around synchronised GPU work, particles resident in HBM).
The equal-error point: the plain sweep (factor-2 steps in K) is refined by
bisection in K until a plain run's error is within 10 % of the learned
error, and the plain throughput at the learned error is interpolated
log-log between the nearest plain runs above and below it; the gain is the
learned throughput over that.  The same is done at equal median particle
error at the end of the run, an error that sees the fast phases; every run
also reports the median error of its first step against the plain push with
K_fine substeps.  With base_K > 0 the network corrects the plain push with
base_K substeps instead of the free rotation (its labels are that push's
defect, which shrinks like base_K^-2), and K_fine and K_ref must resolve
errors far below that push's.

Vlasov-Poisson workload (`equal_error_vp`): the beam R ~ N(0, 1) truncated
to |R| < 4, V ~ N(0, 1), N_r cells on [-5, 5], eps = 1e-3, dt = 0.1.  The
6-input network (features plus E^n(R_n)) is trained on self-generated data: a
separate beam (another seed) is run with the plain push at K_data substeps
and, every `collect_every` steps, its particles, their field E^n and the
labels of a K_fine-substep step in that frozen field are collected on the
GPU.  Reference and error metric as above, with the reference run at K_ref.
The labels take K_fine = 12800 substeps here: the CIC field's gradient jumps
at every node, so the plain push converges slowly in K, and at K = 800 its
own frozen-field energy error (median 7e-5 relative) exceeds the 1e-5 drift
bound; a network fitted closely to such labels inherits that error and fails
the check.

The learned push runs with both inference operand types (BF16, the
library's default, and FP16); the results carry the equal-error point of
each (with the check and without it) and a summary of their gains.

Everything here calls the HIP library through its C ABI.
"""
import time

import numpy as np

from . import (EP_FIELD_DUFFING, EP_FIELD_POISSON, EP_MLP_BF16, EP_MLP_FP16, EP_PUSH_LEARNED,
               EP_PUSH_PLAIN, Sim, capi, synth)

DT, EPS, SIGMA = 0.05, 1e-3, 1.5
NORM_INIT = np.array([SIGMA, 100.0, 1.0, 0.0, 1.0, 0.0, 1.0, 0.0])


def _timed_run(sim, steps):
    """Seconds for `steps` Duffing steps after one untimed step (first-use
    allocations and code loading stay out of the timed region; the field is
    autonomous, so the shifted start changes nothing but the clock)."""
    sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
    sim.sync()
    t0 = time.perf_counter()
    sim.step(DT, EPS, EP_FIELD_DUFFING, steps)
    sim.sync()
    return time.perf_counter() - t0


def _rms_history(sim, R0, V0, w, steps, every):
    sim.set_particles(R0, V0, w)
    out = [sim.moments(EPS, EP_FIELD_DUFFING)["rms_radius"]]
    for _ in range(steps // every):
        sim.step(DT, EPS, EP_FIELD_DUFFING, every)
        out.append(sim.moments(EPS, EP_FIELD_DUFFING)["rms_radius"])
    return np.array(out)


def train(sim, n_train, epochs, K_fine, seed=14, init_seed=5, batch=None, lr=3e-3,
          lr_final=1e-5, base_K=0):
    """Train from Glorot-initialised weights; the batch defaults to ~n/512
    (64-aligned, between 1024 and 4096) so that small sets still take enough
    Adam steps.  Small batches and long schedules pay here: at 1e7 samples,
    80 epochs of batch 4096 reach a normalised loss ~2e-4 against ~6e-3 for
    10 epochs of batch 16384, and the fallback rate at tol 1e-5 falls from
    ~20% to ~0.5%.  base_K > 0: the network corrects the plain push with
    base_K substeps (its labels are that push's defect)."""
    if batch is None:
        batch = max(1024, min(4096, (n_train // 512) // 64 * 64))
    R, V, _ = synth.gaussian(n_train, seed=seed, sigma=SIGMA)
    norm = np.append(NORM_INIT, float(base_K))
    capi.ep_mlp_set_weights(sim.ctx, synth.mlp_init(5, 64, 2, seed=init_seed), norm)
    return capi.ep_mlp_train(sim.ctx, R, V, DT, EPS, K_fine, batch, epochs, lr, lr_final, SIGMA)


def _interp_rate(lo, hi, err, key="rms_err"):
    """Plain throughput at the error `err` between two plain runs whose errors
    bracket it, interpolated linearly in log(throughput) against log(error)
    (locally err ~ K^-p and throughput ~ K^-1, both straight lines there)."""
    if hi[key] == lo[key]:
        return hi["particle_steps_per_s"]
    f = (np.log(err) - np.log(lo[key])) / (np.log(hi[key]) - np.log(lo[key]))
    return float(np.exp(np.log(lo["particle_steps_per_s"]) +
                        f * (np.log(hi["particle_steps_per_s"]) -
                             np.log(lo["particle_steps_per_s"]))))


def _refine(plain, run_plain, err, key="rms_err", rel=0.1, max_runs=4):
    """Bisection in log K between the plain runs whose errors `key` bracket
    `err` (appending new runs to `plain`) until one run's error lies within
    +-rel of it, or max_runs runs were added; returns that run or None."""
    for _ in range(max_runs + 1):
        near = [q for q in plain if abs(q[key] / err - 1.0) <= rel]
        if near:
            return min(near, key=lambda q: q["K"])
        above = [q for q in plain if q[key] > err]
        below = [q for q in plain if q[key] <= err]
        if not above or not below or run_plain is None:
            return None
        lo = max(above, key=lambda q: q["K"])
        hi = min((q for q in below if q["K"] > lo["K"]), key=lambda q: q["K"], default=None)
        if hi is None:
            return None
        K = int(round(np.sqrt(lo["K"] * hi["K"])))
        if K <= lo["K"] or K >= hi["K"]:
            return None
        plain.append(run_plain(K))
        plain.sort(key=lambda q: q["K"])
    return None


def _equal_error_point(plain, entry, run_plain=None, key="rms_err"):
    """The plain push at the learned run's error `key`.  The plain sweep is
    refined by bisection in K until a plain run's error is within 10 % of the
    learned error; the gain is the learned throughput over the plain
    throughput interpolated (log-log) at the learned error between the
    nearest plain runs above and below it.  `matched` is the refined run."""
    err = entry[key]
    matched = _refine(plain, run_plain, err, key)
    above = [q for q in plain if q[key] > err]
    below = [q for q in plain if q[key] <= err]
    if not below:
        return {"plain_K": None, "gain": None, "error": key,
                "note": "no plain K in the sweep reached the learned error"}
    hi = min(below, key=lambda q: q["K"])
    lo = max((q for q in above if q["K"] < hi["K"]), key=lambda q: q["K"], default=None)
    rate = hi["particle_steps_per_s"] if lo is None else _interp_rate(lo, hi, err, key)
    res = {"error": key,
           "plain_K_bracket": [None if lo is None else lo["K"], hi["K"]],
           "plain_err_bracket": [None if lo is None else lo[key], hi[key]],
           "plain_particle_steps_per_s": rate,
           "learned_particle_steps_per_s": entry["particle_steps_per_s"],
           "gain": entry["particle_steps_per_s"] / rate,
           "err_learned": err,
           "gain_vs_cheapest_not_worse": entry["particle_steps_per_s"] /
           hi["particle_steps_per_s"]}
    if matched is not None:
        res["matched"] = {"K": matched["K"], "err": matched[key],
                          "particle_steps_per_s": matched["particle_steps_per_s"],
                          "gain": entry["particle_steps_per_s"] /
                          matched["particle_steps_per_s"]}
    return res


PREC_NAMES = {EP_MLP_BF16: "bf16", EP_MLP_FP16: "fp16"}


def _equal_error_points(out, plain, learned, tol=None, run_plain=None):
    """Equal-error points of the learned runs, per precision p:
    "equal_error_<p>" at the drift bound (the first checked run unless tol is
    given) and "equal_error_no_check_<p>"; "gains" collects their gains at
    equal rms-radius error (interpolated to the learned error, see
    _equal_error_point).  "gains_phase" does the same at equal median
    particle error against the reference, an error that, unlike the rms
    radius of a phase-mixed beam, sees the particles' fast phases."""
    for key, gname, suffix in (("rms_err", "gains", ""),
                               ("median_particle_err", "gains_phase", "_phase")):
        if not all(key in q for q in plain + learned):
            continue
        gains = {}
        for name in dict.fromkeys(e["precision"] for e in learned):
            runs = [e for e in learned if e["precision"] == name]
            checked = [e for e in runs if e["drift_tol"] is not None and
                       (tol is None or e["drift_tol"] == tol)]
            g = {}
            if checked:
                pt = _equal_error_point(plain, checked[0], run_plain, key)
                out["equal_error%s_%s" % (suffix, name)] = pt
                g["with_check"] = pt["gain"]
            pt = _equal_error_point(plain, [e for e in runs if e["drift_tol"] is None][0],
                                    run_plain, key)
            out["equal_error%s_no_check_%s" % (suffix, name)] = pt
            g["no_check"] = pt["gain"]
            gains[name] = g
        out[gname] = gains


def equal_error(n_train=4_000_000, n_eval=1_000_000, steps=200, epochs=80, K_fine=800,
                plain_Ks=(25, 50, 100, 200, 400, 800), K_ref=3200, tol=1e-5, K_fb=400,
                seed_eval=15, every=10, precisions=(EP_MLP_BF16, EP_MLP_FP16), lr_final=1e-5,
                base_K=0, project=False, log=None):
    """Returns a dict with the training report, the plain sweep, the learned
    runs (for each inference precision, with the check at tol and without
    it) and the equal-error points (see _equal_error_points).  base_K > 0:
    the network corrects the plain push with base_K substeps; K_fine and K_ref
    must then resolve errors well below that push's (its defect shrinks like
    K^-2).  project: the learned runs project the particles that pass the
    check onto their energy shell (ep_mlp_set_projection)."""
    def say(msg):
        if log:
            log(msg)

    Re, Ve, we = synth.gaussian(n_eval, seed=seed_eval, sigma=SIGMA)
    out = {"workload": {"field": "duffing", "eps": EPS, "dt": DT, "sigma": SIGMA,
                        "n_train": n_train, "n_eval": n_eval, "steps": steps, "K_fine": K_fine,
                        "K_ref": K_ref, "drift_tol": tol, "fallback_substeps": K_fb,
                        "base_substeps": base_K, "epochs": epochs, "projection": project}}
    with Sim(n_eval, substeps=K_ref) as ref:
        hist_ref = _rms_history(ref, Re, Ve, we, steps, every)
        Rr, Vr = ref.particles()
    rms_ref = float(hist_ref[-1])
    out["rms_ref"] = rms_ref
    say("reference K=%d rms %.6f" % (K_ref, rms_ref))
    ns = min(n_eval, 1_000_000)
    with Sim(n_eval, substeps=K_fine) as fine:
        fine.set_particles(Re, Ve, we)
        fine.step(DT, EPS, EP_FIELD_DUFFING, 1)
        R1f, V1f = fine.particles(0, ns)

    def one_step_err(sim):
        """Median error of one step from the evaluation beam against the plain
        push with K_fine substeps (the labels' accuracy)."""
        sim.set_particles(Re, Ve, we)
        sim.step(DT, EPS, EP_FIELD_DUFFING, 1)
        R1, V1 = sim.particles(0, ns)
        return float(np.median(np.hypot(R1 - R1f, V1 - V1f)))

    def run_error(sim):
        hist = _rms_history(sim, Re, Ve, we, steps, every)
        R, V = sim.particles()
        return (float(np.max(np.abs(hist - hist_ref) / hist_ref)),
                float(np.median(np.hypot(R - Rr, V - Vr))))

    def run_plain(K):
        with Sim(n_eval, substeps=K) as s:
            s.set_particles(Re, Ve, we)
            el = _timed_run(s, steps)
            err, perr = run_error(s)
            serr = one_step_err(s)
        q = {"K": K, "particle_steps_per_s": n_eval * steps / el, "rms_err": err,
             "median_particle_err": perr, "one_step_err": serr}
        say("plain K=%d: %.3e particle-steps/s, rms err %.3e" % (K, q["particle_steps_per_s"], err))
        return q

    plain = [run_plain(K) for K in plain_Ks]
    out["plain"] = plain

    with Sim(n_eval, substeps=1) as sim:
        rep = train(sim, n_train, epochs, K_fine, lr_final=lr_final, base_K=base_K)
        out["train"] = rep
        say("trained: loss %.4f -> %.4f in %d steps (%.0f ms)" % (
            rep["loss_first"], rep["loss_last"], rep["steps"], rep["train_ms"]))
        learned = []
        capi.ep_mlp_set_projection(sim.ctx, project)
        for prec, t in [(p_, t_) for p_ in precisions for t_ in (tol, float("inf"))]:
            capi.ep_mlp_set_precision(sim.ctx, prec)
            sim.set_particles(Re, Ve, we)
            capi.ep_set_push_mode(sim.ctx, EP_PUSH_LEARNED, 1e300 if t == float("inf") else t,
                                  K_fb)
            f0 = sim.moments(EPS, EP_FIELD_DUFFING)["n_fallback"]
            el = _timed_run(sim, steps)
            f1 = sim.moments(EPS, EP_FIELD_DUFFING)["n_fallback"]
            # per-kernel times from a separate short run with timing events
            capi.ep_timing_enable(sim.ctx, True)
            sim.step(DT, EPS, EP_FIELD_DUFFING, 20)
            mlp_ms, cnt = capi.ep_timing_get(sim.ctx, "mlp_push")
            fb_ms, _ = capi.ep_timing_get(sim.ctx, "fallback_push")
            base_ms, _ = capi.ep_timing_get(sim.ctx, "base_push")
            capi.ep_timing_enable(sim.ctx, False)
            err, perr = run_error(sim)
            serr = one_step_err(sim)
            learned.append({"precision": PREC_NAMES[prec],
                            "drift_tol": None if t == float("inf") else t,
                            "particle_steps_per_s": n_eval * steps / el, "rms_err": err,
                            "median_particle_err": perr, "one_step_err": serr,
                            "fallback_rate": (f1 - f0) / (n_eval * (steps + 1)),
                            "network_particle_steps_per_s": n_eval * cnt / (mlp_ms / 1e3),
                            "fallback_ms_per_step": fb_ms / cnt,
                            "base_push_ms_per_step": base_ms / cnt})
            say("learned %s tol=%s: %.3e particle-steps/s, rms err %.3e, fallback %.4f" % (
                PREC_NAMES[prec], t, learned[-1]["particle_steps_per_s"], err,
                learned[-1]["fallback_rate"]))
        capi.ep_set_push_mode(sim.ctx, EP_PUSH_PLAIN)
    out["learned"] = learned
    _equal_error_points(out, plain, learned, run_plain=run_plain)
    return out


# ------------------------------------------------------------------ Vlasov-Poisson

VP_DT, VP_EPS, VP_NR = 0.1, 1e-3, 4096
# feature scales (s_in, s_t, s_E), label normalisation set by training, and
# the amplitude-scaled output map (bounded targets for small orbits)
VP_NORM_INIT = np.array([1.0, 100.0, 0.25, 0.0, 1.0, 0.0, 1.0, 1.0])


def _vp_history(sim, R0, V0, w, steps, every, energy=False):
    """rms radius (and with energy, the total energy) every `every` steps."""
    sim.set_particles(R0, V0, w)
    m = sim.moments(VP_EPS, EP_FIELD_POISSON)
    out, en = [m["rms_radius"]], [m["energy"]]
    for _ in range(steps // every):
        sim.step(VP_DT, VP_EPS, EP_FIELD_POISSON, every)
        m = sim.moments(VP_EPS, EP_FIELD_POISSON)
        out.append(m["rms_radius"])
        en.append(m["energy"])
    return (np.array(out), np.array(en)) if energy else np.array(out)


def train_vp(n_data, steps, nr=VP_NR, K_data=400, K_fine=12800, collect_every=10, epochs=40,
             batch=4096, lr=3e-3, lr_final=1e-5, seed=16, init_seed=5, log=None):
    """Self-generated training: plain run of a separate beam, samples collected
    every `collect_every` steps; returns (params, norm, report, n_samples)."""
    R, V, w = synth.gaussian_truncated(n_data, seed=seed)
    with Sim(n_data, n_cells=nr, substeps=K_data) as sim:
        sim.set_particles(R, V, w)
        capi.ep_mlp_set_weights(sim.ctx, synth.mlp_init(6, 64, 2, seed=init_seed), VP_NORM_INIT)
        total = 0
        for lvl in range(steps // collect_every):
            total = capi.ep_mlp_collect(sim.ctx, VP_DT, VP_EPS, K_fine, reset=lvl == 0)
            sim.step(VP_DT, VP_EPS, EP_FIELD_POISSON, collect_every)
        if log:
            log("vp: collected %d samples" % total)
        b = min(batch, max(64, (total // 512) // 64 * 64))
        rep = capi.ep_mlp_train(sim.ctx, None, None, VP_DT, VP_EPS, K_fine, b, epochs, lr,
                                lr_final, 1.0, field=EP_FIELD_POISSON)
        p, norm = capi.ep_mlp_get_weights(sim.ctx, capi.mlp_n_params(6))
    return p, norm, rep, total


def equal_error_vp(n_eval=1_000_000, n_data=500_000, steps=200, nr=VP_NR, epochs=40,
                   K_fine=12800, plain_Ks=(25, 50, 100, 200, 400, 800), K_ref=3200, tol=1e-5,
                   extra_tols=(1e-4, 1e-3), K_fb=400, seed_eval=17, every=10,
                   precisions=(EP_MLP_BF16, EP_MLP_FP16), single_run=False, n_sample=1_000_000,
                   project=False, log=None):
    """As equal_error, for the Vlasov-Poisson beam; the learned push runs, for
    each precision, at the drift bound tol (the equal-error point), at
    extra_tols and without the check.  With single_run (the at-scale
    workload, where every run is long) each scheme's rate comes from the run
    that records its rms radius (a moments call every `every` steps, < 1 % of
    the step time at 1e8 particles) instead of a run of its own.  Every run
    also reports its energy drift, the median particle error of the first
    n_sample particles at the end against the reference, and the median error
    of its first step (same start, same frozen field) against the plain push
    with K_fine substeps, the labels' own accuracy.  project: as in
    equal_error."""
    def say(msg):
        if log:
            log(msg)

    Re, Ve, we = synth.gaussian_truncated(n_eval, seed=seed_eval)
    ns = min(n_sample, n_eval)
    out = {"workload": {"field": "poisson", "eps": VP_EPS, "dt": VP_DT, "n_cells": nr,
                        "n_eval": n_eval, "n_data": n_data, "steps": steps, "K_fine": K_fine,
                        "K_ref": K_ref, "drift_tol": tol, "fallback_substeps": K_fb,
                        "recorded_every": every, "projection": project}}
    with Sim(n_eval, n_cells=nr, substeps=K_ref) as ref:
        hist_ref, e_ref = _vp_history(ref, Re, Ve, we, steps, every, energy=True)
        Rr, Vr = ref.particles(0, ns)
    out["rms_ref"] = float(hist_ref[-1])
    out["reference_energy_drift"] = float(abs(e_ref[-1] / e_ref[0] - 1))
    say("vp reference K=%d rms %.6f" % (K_ref, hist_ref[-1]))
    with Sim(n_eval, n_cells=nr, substeps=K_fine) as fine:
        fine.set_particles(Re, Ve, we)
        fine.step(VP_DT, VP_EPS, EP_FIELD_POISSON, 1)
        R1f, V1f = fine.particles(0, ns)
    step_errs = {}

    def measured(sim):
        """(seconds, rms-radius error, energy drift, median particle error);
        timed apart from the recording run unless single_run.  Records the
        first step's error in step_errs["last"]."""
        sim.set_particles(Re, Ve, we)
        sim.step(VP_DT, VP_EPS, EP_FIELD_POISSON, 1)   # field and tables ready
        R1, V1 = sim.particles(0, ns)
        step_errs["last"] = float(np.median(np.hypot(R1 - R1f, V1 - V1f)))
        el = None if single_run else timed(sim)
        sim.sync()
        t0 = time.perf_counter()
        h, e = _vp_history(sim, Re, Ve, we, steps, every, energy=True)
        sim.sync()
        if single_run:
            el = time.perf_counter() - t0
        R, V = sim.particles(0, ns)
        return (el, float(np.max(np.abs(h - hist_ref) / hist_ref)), float(abs(e[-1] / e[0] - 1)),
                float(np.median(np.hypot(R - Rr, V - Vr))))

    def timed(sim):
        sim.set_particles(Re, Ve, we)
        sim.step(VP_DT, VP_EPS, EP_FIELD_POISSON, 1)   # field and tables ready
        sim.set_particles(Re, Ve, we)
        sim.sync()
        t0 = time.perf_counter()
        sim.step(VP_DT, VP_EPS, EP_FIELD_POISSON, steps)
        sim.sync()
        return time.perf_counter() - t0

    def run_plain(K):
        with Sim(n_eval, n_cells=nr, substeps=K) as s:
            el, err, drift, perr = measured(s)
        q = {"K": K, "particle_steps_per_s": n_eval * steps / el, "rms_err": err,
             "energy_drift": drift, "median_particle_err": perr,
             "one_step_err": step_errs["last"]}
        say("vp plain K=%d: %.3e particle-steps/s, rms err %.3e" % (K, q["particle_steps_per_s"], err))
        return q

    plain = [run_plain(K) for K in plain_Ks]
    out["plain"] = plain

    # the same number of collected time levels (20) whatever the run length
    p, norm, rep, n_samples = train_vp(n_data, steps, nr=nr, K_fine=K_fine, epochs=epochs,
                                       collect_every=max(10, steps // 20), log=log)
    rep["n_samples"] = n_samples
    out["train"] = rep
    say("vp trained on %d samples: loss %.4f -> %.4f in %d steps (%.0f ms)" % (
        n_samples, rep["loss_first"], rep["loss_last"], rep["steps"], rep["train_ms"]))
    learned = []
    with Sim(n_eval, n_cells=nr, substeps=1) as sim:
        capi.ep_mlp_set_weights(sim.ctx, p, norm)
        capi.ep_mlp_set_projection(sim.ctx, project)
        tols = (tol,) + tuple(extra_tols) + (float("inf"),)
        for prec, t in [(p_, t_) for p_ in precisions for t_ in tols]:
            capi.ep_mlp_set_precision(sim.ctx, prec)
            capi.ep_set_push_mode(sim.ctx, EP_PUSH_LEARNED, 1e300 if t == float("inf") else t,
                                  K_fb)
            sim.set_particles(Re, Ve, we)
            f0 = sim.moments(VP_EPS, EP_FIELD_POISSON)["n_fallback"]
            el, err, drift, perr = measured(sim)
            f1 = sim.moments(VP_EPS, EP_FIELD_POISSON)["n_fallback"]
            # per-kernel times from a separate short run with timing events
            capi.ep_timing_enable(sim.ctx, True)
            sim.step(VP_DT, VP_EPS, EP_FIELD_POISSON, 20)
            mlp_ms, cnt = capi.ep_timing_get(sim.ctx, "mlp_push")
            fb_ms, _ = capi.ep_timing_get(sim.ctx, "fallback_push")
            capi.ep_timing_enable(sim.ctx, False)
            runs = steps + 1 if single_run else 2 * steps + 2
            learned.append({"precision": PREC_NAMES[prec],
                            "drift_tol": None if t == float("inf") else t,
                            "particle_steps_per_s": n_eval * steps / el, "rms_err": err,
                            "energy_drift": drift, "median_particle_err": perr,
                            "one_step_err": step_errs["last"],
                            "fallback_rate": (f1 - f0) / (n_eval * runs),
                            "network_ms_per_step": mlp_ms / cnt,
                            "fallback_ms_per_step": fb_ms / cnt,
                            "network_particle_steps_per_s": n_eval * cnt / (mlp_ms / 1e3)})
            say("vp learned %s tol=%s: %.3e particle-steps/s, rms err %.3e, fallback %.4f" % (
                PREC_NAMES[prec], t, learned[-1]["particle_steps_per_s"], err,
                learned[-1]["fallback_rate"]))
    out["learned"] = learned
    _equal_error_points(out, plain, learned, tol, run_plain=run_plain)
    return out


def long_time_vp(n_eval=10_000_000, steps=10_000, every=100, nr=VP_NR, K_ref=1600,
                 plain_Ks=(100, 200), tol=1e-5, K_fb=400, n_data=10_000_000, epochs=4,
                 precisions=(EP_MLP_FP16, EP_MLP_BF16), seed_eval=17, n_sample=1_000_000,
                 projections=(False, True), log=None):
    """Long-time run of the Vlasov-Poisson beam (eps = 1e-3, dt = 0.1, to
    t = steps dt): the learned push with the drift check against plain runs
    and a plain reference at K_ref, all from the same particles.  Every
    `every` steps: the rms radius (its relative error against the
    reference), the total energy (its drift from t = 0) and, for the learned
    runs, the fallback rate of the interval; at the end, the median particle
    error of the first n_sample particles against the reference.  The network
    is trained on samples collected over the same time span from a separate
    beam of n_data particles (as many as the evaluation beam: the field of a
    smaller beam is noisier, and a network trained on it carries a larger
    bias), and runs with each energy-projection setting in `projections`.
    Rates are timed on runs of their own, without the moment calls."""
    def say(msg):
        if log:
            log(msg)

    R0, V0, w = synth.gaussian_truncated(n_eval, seed=seed_eval)
    ns = min(n_sample, n_eval)
    out = {"workload": {"field": "poisson", "eps": VP_EPS, "dt": VP_DT, "n_cells": nr,
                        "n_eval": n_eval, "steps": steps, "t_end": steps * VP_DT,
                        "K_ref": K_ref, "drift_tol": tol, "fallback_substeps": K_fb}}
    end = {}

    def history(sim, learned):
        sim.set_particles(R0, V0, w)
        m0 = sim.moments(VP_EPS, EP_FIELD_POISSON)
        rms, energy, fb = [m0["rms_radius"]], [m0["energy"]], []
        f_prev = m0["n_fallback"]
        for _ in range(steps // every):
            sim.step(VP_DT, VP_EPS, EP_FIELD_POISSON, every)
            m = sim.moments(VP_EPS, EP_FIELD_POISSON)
            rms.append(m["rms_radius"])
            energy.append(m["energy"])
            if learned:
                fb.append((m["n_fallback"] - f_prev) / (n_eval * every))
                f_prev = m["n_fallback"]
        end["R"], end["V"] = sim.particles(0, ns)
        return np.array(rms), np.array(energy), np.array(fb)

    def rate(sim, n_steps):
        sim.set_particles(R0, V0, w)
        sim.step(VP_DT, VP_EPS, EP_FIELD_POISSON, 1)
        sim.set_particles(R0, V0, w)
        sim.sync()
        t0 = time.perf_counter()
        sim.step(VP_DT, VP_EPS, EP_FIELD_POISSON, n_steps)
        sim.sync()
        return n_eval * n_steps / (time.perf_counter() - t0)

    with Sim(n_eval, n_cells=nr, substeps=K_ref) as ref:
        rms_ref, e_ref, _ = history(ref, False)
    Rr, Vr = end["R"], end["V"]
    say("long-time reference K=%d done" % K_ref)

    def summary(rms, energy):
        err = np.abs(rms - rms_ref) / rms_ref
        drift = np.abs(energy - energy[0]) / abs(energy[0])
        return {"rms_err_max": float(err.max()), "rms_err_final": float(err[-1]),
                "energy_drift_max": float(drift.max()), "energy_drift_final": float(drift[-1]),
                "median_particle_err_final": float(np.median(np.hypot(end["R"] - Rr,
                                                                      end["V"] - Vr)))}

    out["reference"] = {"K": K_ref, **{k: v for k, v in summary(rms_ref, e_ref).items()
                                      if k.startswith("energy")}}
    plain = []
    for K in plain_Ks:
        with Sim(n_eval, n_cells=nr, substeps=K) as sim:
            rms, energy, _ = history(sim, False)
            entry = {"K": K, "particle_steps_per_s": rate(sim, min(steps, 200)),
                     **summary(rms, energy)}
        plain.append(entry)
        say("long-time plain K=%d: %s" % (K, entry))
    out["plain"] = plain
    p, norm, rep, total = train_vp(n_data, steps, nr=nr, collect_every=max(1, steps // 20),
                                   epochs=epochs)
    out["train"] = {"n_samples": total, "loss_first": rep["loss_first"],
                    "loss_last": rep["loss_last"]}
    learned = []
    with Sim(n_eval, n_cells=nr, substeps=1) as sim:
        capi.ep_mlp_set_weights(sim.ctx, p, norm)
        capi.ep_set_push_mode(sim.ctx, EP_PUSH_LEARNED, tol, K_fb)
        for prec, proj in [(p_, q_) for q_ in projections for p_ in precisions]:
            capi.ep_mlp_set_precision(sim.ctx, prec)
            capi.ep_mlp_set_projection(sim.ctx, proj)
            rms, energy, fb = history(sim, True)
            entry = {"precision": PREC_NAMES[prec], "drift_tol": tol, "projection": proj,
                     "particle_steps_per_s": rate(sim, min(steps, 200)),
                     **summary(rms, energy),
                     "fallback_rate_first": float(fb[0]), "fallback_rate_last": float(fb[-1]),
                     "fallback_rate_mean": float(fb.mean())}
            learned.append(entry)
            say("long-time learned %s: %s" % (PREC_NAMES[prec], entry))
    out["learned"] = learned
    return out


def long_time_duffing(n_eval=1_000_000, steps=20_000, every=1000, K_ref=6400,
                      plain_Ks=(800, 1600), base_K=200, n_train=10_000_000, epochs=240,
                      K_fine=6400, tol=1e-5, K_fb=3200, precisions=(EP_MLP_BF16, EP_MLP_FP16),
                      seed_eval=15, n_sample=1_000_000, projections=(False, True), log=None):
    """Long-time run of the Duffing workload (eps = 1e-3, dt = 0.05, R, V ~
    N(0, 1.5), to t = steps dt) with the base-push network (trained as in
    equal_error with base_K) against plain runs and a plain reference at
    K_ref, all from the same particles: every `every` steps the relative
    rms-radius error against the reference and the Duffing energy's drift
    from t = 0, at the end the median particle error of the first n_sample
    particles against the reference; the fallback push (K_fb = 3200) is more
    accurate than the network's step, which matches the plain push at about
    2 000 substeps; the learned runs with each
    energy-projection setting in `projections`.  Rates are timed on runs of
    their own (`every` steps after one untimed step)."""
    def say(msg):
        if log:
            log(msg)

    R0, V0, w = synth.gaussian(n_eval, seed=seed_eval, sigma=SIGMA)
    ns = min(n_sample, n_eval)
    out = {"workload": {"field": "duffing", "eps": EPS, "dt": DT, "sigma": SIGMA,
                        "n_eval": n_eval, "steps": steps, "t_end": steps * DT, "K_ref": K_ref,
                        "base_substeps": base_K, "K_fine": K_fine, "drift_tol": tol,
                        "fallback_substeps": K_fb}}
    end = {}

    def history(sim):
        sim.set_particles(R0, V0, w)
        m = sim.moments(EPS, EP_FIELD_DUFFING)
        rms, energy = [m["rms_radius"]], [m["energy"]]
        for _ in range(steps // every):
            sim.step(DT, EPS, EP_FIELD_DUFFING, every)
            m = sim.moments(EPS, EP_FIELD_DUFFING)
            rms.append(m["rms_radius"])
            energy.append(m["energy"])
        end["R"], end["V"] = sim.particles(0, ns)
        return np.array(rms), np.array(energy)

    def rate(sim):
        sim.set_particles(R0, V0, w)
        return n_eval * every / _timed_run(sim, every)

    with Sim(n_eval, substeps=K_ref) as ref:
        rms_ref, e_ref = history(ref)
    Rr, Vr = end["R"], end["V"]
    say("long-time Duffing reference K=%d done" % K_ref)

    def summary(rms, energy):
        err = np.abs(rms - rms_ref) / rms_ref
        drift = np.abs(energy - energy[0]) / abs(energy[0])
        return {"rms_err_max": float(err.max()), "rms_err_final": float(err[-1]),
                "energy_drift_max": float(drift.max()), "energy_drift_final": float(drift[-1]),
                "median_particle_err_final": float(np.median(np.hypot(end["R"] - Rr,
                                                                      end["V"] - Vr)))}

    drift_ref = np.abs(e_ref - e_ref[0]) / abs(e_ref[0])
    out["reference"] = {"K": K_ref, "energy_drift_max": float(drift_ref.max())}
    plain = []
    for K in plain_Ks:
        with Sim(n_eval, substeps=K) as sim:
            entry = {"K": K, **summary(*history(sim)), "particle_steps_per_s": rate(sim)}
        plain.append(entry)
        say("long-time Duffing plain K=%d: %s" % (K, entry))
    out["plain"] = plain
    learned = []
    with Sim(n_eval, substeps=1) as sim:
        rep = train(sim, n_train, epochs, K_fine, lr_final=1e-6, base_K=base_K)
        out["train"] = {"loss_first": rep["loss_first"], "loss_last": rep["loss_last"]}
        for prec, proj in [(p_, q_) for q_ in projections for p_ in precisions]:
            capi.ep_mlp_set_precision(sim.ctx, prec)
            capi.ep_mlp_set_projection(sim.ctx, proj)
            capi.ep_set_push_mode(sim.ctx, EP_PUSH_LEARNED, tol, K_fb)
            sim.set_particles(R0, V0, w)
            f0 = sim.moments(EPS, EP_FIELD_DUFFING)["n_fallback"]
            entry = {"precision": PREC_NAMES[prec], "drift_tol": tol, "projection": proj,
                     **summary(*history(sim))}
            f1 = sim.moments(EPS, EP_FIELD_DUFFING)["n_fallback"]
            entry["fallback_rate"] = (f1 - f0) / (n_eval * steps)
            entry["particle_steps_per_s"] = rate(sim)
            learned.append(entry)
            say("long-time Duffing learned %s: %s" % (PREC_NAMES[prec], entry))
        capi.ep_set_push_mode(sim.ctx, EP_PUSH_PLAIN)
    out["learned"] = learned
    return out


# ------------------------------------------------------------ the paper's own schemes

def _run_scheme(R0, V0, w, field, mode, dt, eps, steps, nr=VP_NR, substeps=1, h_fine=0.0,
                periods_once=True):
    """Returns (R, V, seconds, extra) after `steps` macro steps of `mode`.
    One untimed step of a small subset in a context of its own first takes
    the first-launch costs out of the timing."""
    m = min(R0.size, 1024)
    with Sim(m, n_cells=nr, substeps=substeps) as warm:
        warm.set_particles(R0[:m], V0[:m], w * R0.size / m)
        capi.ep_set_push_mode(warm.ctx, mode)
        capi.ep_set_fine_solver(warm.ctx, h_fine, periods_once=periods_once)
        warm.step(dt, eps, field, 1)
        warm.sync()
    with Sim(R0.size, n_cells=nr, substeps=substeps) as sim:
        sim.set_particles(R0, V0, w)
        capi.ep_set_push_mode(sim.ctx, mode)
        capi.ep_set_fine_solver(sim.ctx, h_fine, periods_once=periods_once)
        sim.sync()
        t0 = time.perf_counter()
        sim.step(dt, eps, field, steps)
        sim.sync()
        el = time.perf_counter() - t0
        extra = {}
        if mode == capi.EP_PUSH_IMPROVED_ETD:
            T, N, un = capi.ep_get_periods(sim.ctx, R0.size)
            extra = {"N_median": float(np.median(N)), "N_min": int(N.min()),
                     "N_max": int(N.max()), "unresolved": un}
        R, V = sim.particles()
    return R, V, el, extra


def paper_schemes(n_duffing=1_000_000, n_vp=100_000, eps=1e-3, dt=0.5, steps_duffing=20,
                  steps_vp=4, plain_K=(100, 400), nr=1024, ref_refine=4, log=None):
    """The improved ETD scheme (Algorithm 3.4; for Duffing both with the
    periods found at the first step, as the paper does, and searched at every
    step), the classic and modified ETD schemes (Algorithm 2.1) and the plain
    exponential integrator against the paper's reference solver (RK4, field
    re-solved at every stage) on the paper's initial beam (eq. 2.7), eps = 1e-3, dt = 0.5:
    particle-steps/s (macro steps) and, at the end against the reference, the
    relative rms-radius and median particle errors, which include the fast
    phase, and two errors of the moduli |y|, which do not: the relative
    error of their rms and the mean distance between the sorted moduli
    (relative to their mean).  The reference runs
    with ref_refine times the paper's fine resolution (step 2 pi eps /
    (100 ref_refine)): at 2 pi eps / 100 its own phase error, ~1e-4 per unit
    time at eps = 1e-3, would exceed the errors being measured.  The rate of
    the reference at the paper's step is reported too."""
    def say(msg):
        if log:
            log(msg)

    out = {}
    for field, name, n, steps in ((EP_FIELD_DUFFING, "duffing", n_duffing, steps_duffing),
                                  (EP_FIELD_POISSON, "poisson", n_vp, steps_vp)):
        R0, V0, w = synth.paper_f0(n, seed=18)
        h_ref = 2.0 * np.pi * eps / (100.0 * ref_refine)
        Rr, Vr, el_ref, _ = _run_scheme(R0, V0, w, field, capi.EP_PUSH_RK4, dt, eps, steps, nr,
                                        h_fine=h_ref)
        _, _, el_paper, _ = _run_scheme(R0, V0, w, field, capi.EP_PUSH_RK4, dt, eps, 1, nr)
        rms_ref = float(np.sqrt(np.mean(Rr ** 2)))
        res = {"n": n, "steps": steps, "t_end": steps * dt, "eps": eps, "dt": dt,
               "reference": {"scheme": "RK4, step 2 pi eps/%d, field per stage" % (100 * ref_refine),
                             "particle_steps_per_s": n * steps / el_ref},
               "rk4_at_paper_step": {"scheme": "RK4, step 2 pi eps/100, field per stage",
                                     "particle_steps_per_s": n / el_paper}}

        mod_ref = np.sort(np.hypot(Rr, Vr))
        rms_mod_ref = float(np.sqrt(np.mean(mod_ref ** 2)))

        def score(R, V, el):
            # the moduli |y| barely change over one fast rotation: their
            # distribution measures the slow dynamics whatever the particles'
            # fast phases, which the rms radius and the particle errors mix in
            mod = np.sort(np.hypot(R, V))
            return {"particle_steps_per_s": n * steps / el,
                    "rms_err": abs(float(np.sqrt(np.mean(R ** 2))) - rms_ref) / rms_ref,
                    "median_particle_err": float(np.median(np.hypot(R - Rr, V - Vr))),
                    "rms_modulus_err": abs(float(np.sqrt(np.mean(mod ** 2))) - rms_mod_ref)
                    / rms_mod_ref,
                    "modulus_distribution_err": float(np.mean(np.abs(mod - mod_ref))
                                                      / np.mean(mod_ref))}

        R, V, el, extra = _run_scheme(R0, V0, w, field, capi.EP_PUSH_IMPROVED_ETD, dt, eps, steps,
                                      nr)
        res["improved_etd"] = dict(score(R, V, el), **extra)
        if field == EP_FIELD_DUFFING:
            # the periods searched again at every step instead of found once
            R, V, el, extra = _run_scheme(R0, V0, w, field, capi.EP_PUSH_IMPROVED_ETD, dt, eps,
                                          steps, nr, periods_once=False)
            res["improved_etd_search_every_step"] = dict(score(R, V, el), **extra)
        for name_m, mode in (("classic_etd", capi.EP_PUSH_CLASSIC_ETD),
                             ("modified_etd", capi.EP_PUSH_MODIFIED_ETD)):
            R, V, el, _ = _run_scheme(R0, V0, w, field, mode, dt, eps, steps, nr)
            res[name_m] = score(R, V, el)
        for K in plain_K:
            R, V, el, _ = _run_scheme(R0, V0, w, field, capi.EP_PUSH_PLAIN, dt, eps, steps, nr,
                                      substeps=K)
            res["plain_K%d" % K] = score(R, V, el)
        say("%s: reference %.3e, improved ETD %.3e particle-steps/s (rms err %.2e)" % (
            name, res["reference"]["particle_steps_per_s"],
            res["improved_etd"]["particle_steps_per_s"], res["improved_etd"]["rms_err"]))
        out[name] = res
    return out


def paper_schemes_long(n=100_000, eps_values=(1e-3, 1e-4), dt=0.5, t_end=90.0,
                       checkpoints=(10.0, 30.0, 60.0, 90.0), plain_K=400, ref_refine=4,
                       log=None):
    """The paper's schemes over its long runs in the given (Duffing) field:
    the paper's beam (eq. 2.7), dt = 0.5 to t = 90, eps = 1e-3 and 1e-4.  At
    each checkpoint time every scheme's particles are compared with the
    reference RK4 (step 2 pi eps / (100 ref_refine)): the median particle
    error and the modulus-distribution error (mean distance between the
    sorted moduli |y|, relative to their mean), null once a scheme has blown
    up.  Rates are whole-run particle-steps/s."""
    def say(msg):
        if log:
            log(msg)

    R0, V0, w = synth.paper_f0(n, seed=18)
    marks = [int(round(t / dt)) for t in checkpoints if t <= t_end + 1e-9]
    out = {"n": n, "dt": dt, "t_end": t_end, "checkpoints": [m * dt for m in marks]}

    def run(mode, eps, h_fine=0.0, substeps=1):
        snaps, elapsed, done = [], 0.0, 0
        with Sim(n, n_cells=VP_NR, substeps=substeps) as sim:
            sim.set_particles(R0, V0, w)
            capi.ep_set_push_mode(sim.ctx, mode)
            capi.ep_set_fine_solver(sim.ctx, h_fine)
            for m in marks:
                sim.sync()
                t0 = time.perf_counter()
                sim.step(dt, eps, EP_FIELD_DUFFING, m - done)
                sim.sync()
                elapsed += time.perf_counter() - t0
                done = m
                snaps.append(sim.particles())
        return snaps, n * done / elapsed

    for eps in eps_values:
        h_ref = 2.0 * np.pi * eps / (100.0 * ref_refine)
        ref, rate_ref = run(capi.EP_PUSH_RK4, eps, h_fine=h_ref)
        res = {"reference": {"scheme": "RK4, step 2 pi eps/%d" % (100 * ref_refine),
                             "particle_steps_per_s": rate_ref}}
        schemes = (("improved_etd", capi.EP_PUSH_IMPROVED_ETD, 1),
                   ("classic_etd", capi.EP_PUSH_CLASSIC_ETD, 1),
                   ("modified_etd", capi.EP_PUSH_MODIFIED_ETD, 1),
                   ("plain_K%d" % plain_K, capi.EP_PUSH_PLAIN, plain_K))
        for name, mode, K in schemes:
            snaps, rate = run(mode, eps, substeps=K)
            med, modd = [], []
            def finite(x):   # null in the JSON line once a scheme has blown up
                return float(x) if np.isfinite(x) else None

            for (R, V), (Rr, Vr) in zip(snaps, ref):
                med.append(finite(np.median(np.hypot(R - Rr, V - Vr))))
                mod, mod_ref = np.sort(np.hypot(R, V)), np.sort(np.hypot(Rr, Vr))
                modd.append(finite(np.mean(np.abs(mod - mod_ref)) / np.mean(mod_ref)))
            res[name] = {"particle_steps_per_s": rate, "median_particle_err": med,
                         "modulus_distribution_err": modd}
            say("eps %g %s: %.3e particle-steps/s, median err %s" % (
                eps, name, rate, " ".join("nan" if x is None else "%.2e" % x for x in med)))
        out["eps_%g" % eps] = res
    return out


def paper_schemes_long_vp(runs=((1e-3, 60.0, (10.0, 30.0, 60.0)),), n=20_000, nr=256, dt=0.5,
                          plain_Ks=(100, 400), log=None):
    """The paper's self-consistent long runs (section 4.2): its beam
    (eq. 2.7) with N_p = 20000 macroparticles and the Poisson field on 256
    cells, dt = 0.5, for each (eps, t_end, checkpoint times) of `runs` (the
    paper's are eps = 1e-3 to t = 60 and eps = 1e-4 to t = 90).  The
    reference is its RK4 solver at its own step 2 pi eps / 100 with the field
    re-solved at every stage; the improved ETD scheme (Algorithm 3.4, periods
    searched at every macro step, fine solves with the field per stage), the
    classic ETD scheme (Algorithm 2.1) and the plain exponential integrator
    (field frozen over each macro step) are compared with it at every
    checkpoint: median particle error, modulus-distribution error (mean
    distance between the sorted moduli |y|, relative to their mean: the slow
    dynamics, independent of the fast phases) and relative rms-radius error;
    null once a scheme has blown up.  Rates are whole-run particle-steps/s."""
    def say(msg):
        if log:
            log(msg)

    R0, V0, w = synth.paper_f0(n, seed=18)
    out = {"n": n, "n_cells": nr, "dt": dt}

    def finite(x):
        return float(x) if np.isfinite(x) else None

    for eps, t_end, checkpoints in runs:
        marks = [int(round(t / dt)) for t in checkpoints if t <= t_end + 1e-9]

        def run(mode, substeps=1):
            snaps, elapsed, done = [], 0.0, 0
            with Sim(n, n_cells=nr, substeps=substeps) as sim:
                sim.set_particles(R0, V0, w)
                capi.ep_set_push_mode(sim.ctx, mode)
                capi.ep_set_fine_solver(sim.ctx, 0.0)
                for m in marks:
                    sim.sync()
                    t0 = time.perf_counter()
                    sim.step(dt, eps, EP_FIELD_POISSON, m - done)
                    sim.sync()
                    elapsed += time.perf_counter() - t0
                    done = m
                    snaps.append(sim.particles())
                    say("vp long eps %g mode %d K %d: t = %g" % (eps, mode, substeps, m * dt))
            return snaps, n * done / elapsed

        ref, rate_ref = run(capi.EP_PUSH_RK4)
        res = {"t_end": t_end, "checkpoints": [m * dt for m in marks],
               "reference": {"scheme": "RK4, step 2 pi eps/100, field per stage",
                             "particle_steps_per_s": rate_ref,
                             "rms_radius": [float(np.sqrt(np.mean(R ** 2))) for R, _ in ref]}}
        schemes = [("improved_etd", capi.EP_PUSH_IMPROVED_ETD, 1),
                   ("classic_etd", capi.EP_PUSH_CLASSIC_ETD, 1)]
        schemes += [("plain_K%d" % K, capi.EP_PUSH_PLAIN, K) for K in plain_Ks]
        for name, mode, K in schemes:
            snaps, rate = run(mode, substeps=K)
            med, modd, rms = [], [], []
            for (R, V), (Rr, Vr) in zip(snaps, ref):
                med.append(finite(np.median(np.hypot(R - Rr, V - Vr))))
                mod, mod_ref = np.sort(np.hypot(R, V)), np.sort(np.hypot(Rr, Vr))
                modd.append(finite(np.mean(np.abs(mod - mod_ref)) / np.mean(mod_ref)))
                rr = np.sqrt(np.mean(Rr ** 2))
                rms.append(finite(abs(np.sqrt(np.mean(R ** 2)) - rr) / rr))
            res[name] = {"particle_steps_per_s": rate, "median_particle_err": med,
                         "modulus_distribution_err": modd, "rms_err": rms}
            say("vp long eps %g %s: %.3e particle-steps/s, median err %s, modulus err %s" % (
                eps, name, rate, " ".join("nan" if x is None else "%.2e" % x for x in med),
                " ".join("nan" if x is None else "%.2e" % x for x in modd)))
        out["eps_%g" % eps] = res
    return out


def period_diagnostics(n=100_000, eps=0.01, t_end=5.0, dt=0.05, K=4, nr=1024):
    """The paper's period and modulus diagnostics (section 2) on its initial
    beam (eq. 2.7) at eps = 0.01: the Duffing periods against 2 pi eps, and in
    the self-consistent field the periods and moduli at t_end (plain push)
    against those at t = 0."""
    from . import diagnostics
    R0, V0, w = synth.paper_f0(n, seed=19)
    out = {"n": n, "eps": eps}
    with Sim(n, n_cells=nr, substeps=K) as sim:
        sim.set_particles(R0, V0, w)
        d, _ = diagnostics.period_summary(sim, eps, EP_FIELD_DUFFING)
        out["duffing_periods"] = {k: v for k, v in d.items() if "histogram" not in k and "edges" not in k}
        sim.set_particles(R0, V0, w)
        d0, T0 = diagnostics.period_summary(sim, eps, EP_FIELD_POISSON)
        sim.step(dt, eps, EP_FIELD_POISSON, int(round(t_end / dt)))
        d1, T1 = diagnostics.period_summary(sim, eps, EP_FIELD_POISSON)
        R, V = sim.particles()
    out["poisson_periods_t0"] = {k: v for k, v in d0.items() if "histogram" not in k and "edges" not in k}
    out["poisson_periods_t_end"] = {k: v for k, v in d1.items() if "histogram" not in k and "edges" not in k}
    out["poisson_period_change"] = diagnostics.period_change(T0, T1)
    out["poisson_modulus_change"] = diagnostics.modulus_change(R0, V0, R, V)
    out["t_end"] = t_end
    return out
