"""Benchmark: particle-steps/s of the exponential-integrator PIC step on one MI355X.

Workload (default): the Vlasov-Poisson beam at scale -- N_p = 1e8 FP32
particles, R ~ N(0,1) truncated to |R| < 4, V ~ N(0,1), weights 1/N_p, radial
mesh of N_r = 4096 cells on [-5, 5], eps = 1e-3, dt = 0.05, K = 1 substep,
LDS-privatised fixed-point deposit.  One step = gather + push + CIC deposit (one
fused kernel) and the exact-integer prefix-sum Poisson solve for the next step
(one workgroup); FP64 phase tables per chunk of steps; moments every 100 steps.

Output: one JSON line (see the repository's documentation for the fields),
with
  roofline     -- dominant kernel (push_poisson for the atomic deposit),
                  algorithmic bytes per launch (16 B per particle) / its mean
                  duration from HIP events recorded on the library's stream
                  around every launch, vs the 8 TB/s HBM peak;
  kernels      -- every kernel of the step with its mean duration;
  deposit_comparison -- a short run with the other deposit (sort-by-cell
                  segmented reduction vs LDS-privatised atomics);
  cpu_baseline -- the FP64 CPU oracle timed on this host on a bounded sample;
  learned_vs_plain -- the equal-error comparison of the learned corrector
                  (BF16 and FP16 inference, with the 1e-5 check and without)
                  (Duffing field, eps = 1e-3, dt = 0.05, trained on 1e7
                  samples, evaluated on 1e7 particles; see
                  paper_1404_1160_amd/compare.py);
  learned_vs_plain_base -- the same with a base push: the network corrects
                  the plain push with K_b substeps (its labels that push's
                  defect against K_fine = 6400 substeps);
  learned_vs_plain_vp -- the same for the Vlasov-Poisson beam (N_r = 4096,
                  eps = 1e-3, dt = 0.1, 6-input network trained on samples
                  self-generated from a plain run of a 1e7-particle beam,
                  evaluated on 1e8 particles over 1e3 steps against the plain
                  push with K_ref = 1600), with the energy projection;
  paper_schemes -- the paper's improved ETD scheme (Algorithm 3.4) and the
                  plain push against its RK4 reference on its initial beam
                  (eq. 2.7), eps = 1e-3, dt = 0.5 (Duffing 1e6 particles,
                  Vlasov-Poisson 1e5).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_PARTICLE_STEP = 16   # read + write zR, zV (FP32)
COUNTERS = os.path.join(ROOT, "profiles", "push_poisson_1e8_nr4096_hbm_counters.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1404_1160_amd", "csrc", f)
                  for f in ("pic_kernels.hip", "pic_device.h", "internal.h")]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--cells", type=int, default=4096)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--dt", type=float, default=0.05)
    ap.add_argument("--substeps", type=int, default=1)
    ap.add_argument("--deposit", choices=["atomic", "sorted"], default="atomic")
    ap.add_argument("--moments-every", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-deposit-comparison", action="store_true",
                    help="skip the short run with the other deposit")
    ap.add_argument("--comparison-steps", type=int, default=50)
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the plain-vs-learned equal-error comparison")
    ap.add_argument("--long-time", action="store_true",
                    help="add the long-time runs: learned Vlasov-Poisson (1e7 particles, "
                         "1e4 steps), learned Duffing with a base push (1e6 particles, 2e4 "
                         "steps), each with and without the energy projection, the learned "
                         "Vlasov-Poisson comparison at 1e8 particles without the projection, "
                         "and the paper's schemes to t = 90; several minutes")
    ap.add_argument("--no-paper-schemes", action="store_true",
                    help="skip the reference-RK4 / improved-ETD measurement")
    ap.add_argument("--learned-train", type=int, default=10_000_000)
    ap.add_argument("--learned-eval", type=int, default=10_000_000)
    ap.add_argument("--learned-vp-data", type=int, default=10_000_000,
                    help="beam size of the self-generated Vlasov-Poisson training run")
    ap.add_argument("--learned-vp-epochs", type=int, default=4,
                    help="training epochs of the Vlasov-Poisson network (4 epochs of the "
                         "default 2e8 samples are 195k Adam steps)")
    ap.add_argument("--learned-vp-eval", type=int, default=100_000_000,
                    help="particles of the learned Vlasov-Poisson comparison")
    ap.add_argument("--learned-vp-steps", type=int, default=1000,
                    help="steps of the learned Vlasov-Poisson comparison")
    ap.add_argument("--learned-base-substeps", type=int, default=200,
                    help="substeps of the plain push that the base-push network corrects "
                         "(Duffing field); 0 skips that comparison")
    return ap.parse_args()


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(n, cells, substeps):
    """HBM bytes per push launch (FETCH_SIZE + WRITE_SIZE, each scaled by the
    same counter's reading for a device copy of known size) from the committed
    rocprofv3 counter summary, or None if it was taken on another version of
    the kernel source or at another size of the workload."""
    fields = {}
    try:
        with open(COUNTERS) as f:
            for line in f:
                key, sep, val = line.strip().partition(": ")
                if sep and key in ("kernel_source_sha256_16", "n_particles", "n_cells",
                                   "substeps", "bytes_per_launch"):
                    fields[key] = val.strip()
    except OSError:
        return None
    if fields.get("kernel_source_sha256_16") != kernel_hash():
        return None
    if (fields.get("n_particles"), fields.get("n_cells"), fields.get("substeps")) != (
            str(n), str(cells), str(substeps)) or "bytes_per_launch" not in fields:
        return None
    return int(fields["bytes_per_launch"])


def device_copy_bandwidth(n):
    """Achieved bandwidth of a plain device copy of the particle state's size
    (8 B per particle read and written), as a practical ceiling beside the
    8 TB/s peak: GB/s counting read plus written bytes.  200 copies (about
    0.3 s at 1e8 particles) measure the steady state rather than the first
    milliseconds of a freshly started device."""
    from paper_1404_1160_amd import capi
    return capi.ep_copy_bandwidth(8 * n, reps=200)


def cpu_baseline(n_full, cells, eps, dt, K, seconds):
    """The FP64 oracle on this host: a 2e6-particle sample of the same beam
    (weights scaled to the full beam's charge), stepped until ~`seconds` on
    all the threads it uses, then a 2e5-particle sample on one thread for
    ~seconds/4."""
    import oracle
    from paper_1404_1160_amd import synth

    def rate(n, budget):
        R, V, _ = synth.gaussian_truncated(n, seed=13)
        w = 1.0 / n
        steps = 0
        t0 = time.perf_counter()
        while True:
            R, V = oracle.run(R, V, w, dt, eps, K, 1, oracle.FIELD_POISSON, nr=cells,
                              rmin=-5.0, rmax=5.0)
            steps += 1
            el = time.perf_counter() - t0
            if el >= budget:
                return n * steps / el, steps, el

    n = min(n_full, 2_000_000)
    cores = oracle.threads()
    value, steps, el = rate(n, seconds)
    n1 = min(n_full, 200_000)
    oracle.set_threads(1)
    try:
        value1, steps1, el1 = rate(n1, seconds / 4)
    finally:
        oracle.set_threads(cores)
    return {"value": value, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "sample": "%d particles of the same beam x %d steps (K=%d, N_r=%d), %.1f s" % (
                n, steps, K, cells, el),
            "single_thread": {"value": value1, "unit": "particle-steps/s", "cores": 1,
                              "sample": "%d particles x %d steps, %.1f s" % (n1, steps1, el1)}}


# algorithmic HBM bytes per particle of each particle kernel (FP32 state and
# u32 ids; the mesh is LDS/L2 resident).  The sort passes of every step but the
# first of a call read the 12-byte (R, V, id) records the scatter writes; the
# first count pass reads 8 B of SoA state, and sort_unpack turns the last
# records back into the SoA state once per call (12 B read, 12 B written).
KERNEL_BYTES = {"push_poisson": 16, "sort_count": 12, "sort_scatter": 24, "sort_unpack": 24}
# HIP events on every 10th launch of each kernel: the averages come from a
# tenth of the timed steps (50 launches of 500, 2 of 20), and the events' own
# cost stays out of the other nine tenths: a dispatch that carries events
# ends with a release that writes back the L2, about 28 us per timed push
# launch, so timing every 5th launch cost 1.9 % of the step
TIMING_STRIDE = 10
STEP_KERNELS = ("push_poisson", "mesh_solve", "potential", "sort_count", "sort_offsets", "sort_scatter",
                "sort_combine", "sort_unpack")


def run_pic(args, deposit, steps, warmup, R0, V0, w, copy_ceiling=None):
    """Time `steps` Poisson steps; returns (particle-steps/s, ms/step, kernel table, moments).
    copy_ceiling: a dict that receives the device-copy bandwidth, measured
    after the particles are loaded and right before the warm-up steps, so
    that ceiling and push see the device in the same state."""
    from paper_1404_1160_amd import EP_DEPOSIT_ATOMIC, EP_DEPOSIT_SORTED, EP_FIELD_POISSON, Sim, capi

    n = R0.size
    dep = EP_DEPOSIT_SORTED if deposit == "sorted" else EP_DEPOSIT_ATOMIC
    sim = Sim(n, n_cells=args.cells, substeps=args.substeps, deposit=dep, device=0)
    sim.sync()
    t_set = time.perf_counter()
    sim.set_particles(R0, V0, w)
    sim.sync()
    t_set = time.perf_counter() - t_set
    if copy_ceiling is not None:
        copy_ceiling["GB_per_s"] = device_copy_bandwidth(n)
    for _ in range(warmup):
        sim.step(args.dt, args.eps, EP_FIELD_POISSON, 1)
    sim.sync()
    capi.ep_timing_enable(sim.ctx, TIMING_STRIDE)
    sim.sync()
    t0 = time.perf_counter()
    done = 0
    mom = None
    while done < steps:
        chunk = min(args.moments_every, steps - done)
        sim.step(args.dt, args.eps, EP_FIELD_POISSON, chunk)
        done += chunk
        if done % args.moments_every == 0:
            mom = sim.moments(args.eps, EP_FIELD_POISSON)
    sim.sync()
    elapsed = time.perf_counter() - t0
    kernels = {}
    for name in STEP_KERNELS:
        ms, cnt = capi.ep_timing_get(sim.ctx, name)
        if cnt:
            k = {"ms_per_launch": ms / cnt, "launches_timed": cnt,
                 "timing_stride": TIMING_STRIDE}
            if name in KERNEL_BYTES:
                k["bytes_per_launch"] = KERNEL_BYTES[name] * n
                k["GB_per_s"] = KERNEL_BYTES[name] * n / (ms / cnt / 1e3) / 1e9
            kernels[name] = k
    if mom is None:
        mom = sim.moments(args.eps, EP_FIELD_POISSON)
    # more steps without the timing events (ep_timing_enable clears the table,
    # read above), for comparison
    capi.ep_timing_enable(sim.ctx, False)
    n_plain = min(steps, 200)
    sim.sync()
    t1 = time.perf_counter()
    sim.step(args.dt, args.eps, EP_FIELD_POISSON, n_plain)
    sim.sync()
    ms_untimed = (time.perf_counter() - t1) / n_plain * 1e3
    t_get = time.perf_counter()
    sim.particles()
    t_get = time.perf_counter() - t_get
    sim.close()
    # host hand-over through the C ABI (FP64 host arrays <-> FP32 device state),
    # outside the timed region: the rate if each run started and ended on the host
    transfer = {"set_particles_s": t_set, "get_particles_s": t_get,
                "pcie_inclusive_particle_steps_per_s": n * steps / (elapsed + t_set + t_get),
                "ms_per_step_without_timing_events": ms_untimed}
    kernels["_transfer"] = transfer
    return n * steps / elapsed, elapsed / steps * 1e3, kernels, mom


# network flops per particle-step of the learned push: 2 (5*64 + 64*64 + 64*2)
# for the 5-input network (Duffing), 2 (6*64 + 64*64 + 64*2) with the field
# feature; dense BF16 and FP16 MFMA peak of the MI355X
LEARNED_FLOPS = {"duffing": 9088, "poisson": 9216}
MFMA_PEAK_TFLOPS = 2500.0


def learned_roofline(line):
    """MFMA roofline of the learned push's network kernel (mlp_push), per
    field and inference operand type: algorithmic network flops per
    particle-step times the kernel's own particle-steps/s (HIP events around
    its launches in the comparison runs), against the dense 16-bit MFMA peak."""
    out = {}
    for key, field in (("learned_vs_plain", "duffing"), ("learned_vs_plain_vp", "poisson")):
        for e in line.get(key, {}).get("learned", []):
            if e["drift_tol"] is not None:
                continue
            rate = e["network_particle_steps_per_s"]
            tf = rate * LEARNED_FLOPS[field] / 1e12
            out["%s_%s" % (field, e["precision"])] = {
                "bound": "mfma", "achieved": tf, "peak": MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tf / MFMA_PEAK_TFLOPS, "traffic": None, "kernel": "mlp_push",
                "flop_per_particle_step": LEARNED_FLOPS[field],
                "network_particle_steps_per_s": rate}
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only; --gpus %d is not supported "
              "(the multi-GPU sharding is a design note, not a run)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    from paper_1404_1160_amd import capi, synth

    capi.lib()   # fails loudly if the HIP library is missing
    n = args.n
    t0 = time.perf_counter()
    R0, V0, w = synth.gaussian_truncated(n, seed=13)
    print("bench: %d particles generated in %.1f s" % (n, time.perf_counter() - t0),
          file=sys.stderr, flush=True)

    ceiling = {}
    value, ms_step, kernels, mom = run_pic(args, args.deposit, args.steps, args.warmup, R0, V0, w,
                                           copy_ceiling=ceiling)
    copy_gbs = ceiling["GB_per_s"]
    transfer = kernels.pop("_transfer")
    bw = {k: v for k, v in kernels.items() if "GB_per_s" in v}
    dom = max(bw, key=lambda k: bw[k]["ms_per_launch"] * bw[k]["launches_timed"])
    achieved = bw[dom]["GB_per_s"]
    traffic = (measured_traffic(n, args.cells, args.substeps) if dom == "push_poisson" else None)
    line = {
        "metric": "particle-steps/s at 1e8 particles (plain push, Vlasov-Poisson)",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "vlasov_poisson_beam_Np%d_Nr%d" % (n, args.cells),
                   "n_particles": n, "n_cells": args.cells, "eps": args.eps, "dt": args.dt,
                   "substeps": args.substeps, "deposit": args.deposit,
                   "moments_every": args.moments_every,
                   "precision": "FP32 particle state; FP64 phase and in-register push "
                                "arithmetic; exact-integer charge scan"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": dom, "kernel_ms": bw[dom]["ms_per_launch"],
                     "launches": args.steps, "launches_timed": bw[dom]["launches_timed"],
                     "timing_stride": TIMING_STRIDE,
                     "bytes_per_launch": bw[dom]["bytes_per_launch"],
                     "traffic_over_algorithmic": (traffic / bw[dom]["bytes_per_launch"]
                                                  if traffic else None),
                     "device_copy_GB_per_s": copy_gbs,
                     "frac_of_device_copy": achieved / copy_gbs},
        "kernels": kernels,
        "host_transfer": transfer,
        "moments": {k: mom[k] for k in ("t", "rms_radius", "energy", "n_offmesh", "n_nan")},
    }
    if not args.no_deposit_comparison:
        # the other eps of the at-scale configuration, same beam and mesh
        other_eps = 1e-2 if args.eps != 1e-2 else 1e-3
        a2 = argparse.Namespace(**vars(args))
        a2.eps = other_eps
        v3, ms3, k3, _ = run_pic(a2, args.deposit, args.comparison_steps, 3, R0, V0, w)
        k3.pop("_transfer")
        line["eps_comparison"] = {"eps": other_eps, "particle_steps_per_s": v3,
                                  "ms_per_step": ms3, "kernels": k3}
        other = "sorted" if args.deposit == "atomic" else "atomic"
        v2, ms2, k2, _ = run_pic(args, other, args.comparison_steps, 3, R0, V0, w)
        k2.pop("_transfer")
        line["deposit_comparison"] = {
            args.deposit: {"particle_steps_per_s": value, "ms_per_step": ms_step},
            other: {"particle_steps_per_s": v2, "ms_per_step": ms2, "kernels": k2}}
    del R0, V0
    if not args.no_learned:
        from paper_1404_1160_amd import compare
        say = lambda m: print("bench: " + m, file=sys.stderr, flush=True)
        print("bench: learned-vs-plain comparison", file=sys.stderr, flush=True)
        line["learned_vs_plain"] = compare.equal_error(
            n_train=args.learned_train, n_eval=args.learned_eval, epochs=240, lr_final=1e-6,
            log=say)
        if args.learned_base_substeps > 0:
            print("bench: learned-vs-plain comparison with a base push of %d substeps"
                  % args.learned_base_substeps, file=sys.stderr, flush=True)
            line["learned_vs_plain_base"] = compare.equal_error(
                n_train=args.learned_train, n_eval=args.learned_eval, epochs=240,
                lr_final=1e-6, K_fine=6400, K_ref=6400, plain_Ks=(200, 400, 800, 1600, 3200),
                base_K=args.learned_base_substeps, K_fb=3200, log=say)
        print("bench: learned-vs-plain comparison, Vlasov-Poisson at scale", file=sys.stderr,
              flush=True)
        # the learned Vlasov-Poisson workload at its size: 1e8 particles,
        # N_r = 4096, eps = 1e-3, dt = 0.1, 1e3 steps (the full 1e5 steps are
        # out of the default run's time), reference plain K = 1600 (the plain
        # push converges slowly in K on the CIC field, whose gradient jumps at
        # every node; every run reports its one-step error against the
        # labels' K_fine = 12800 beside it)
        # with the energy projection (ep_mlp_set_projection), which keeps
        # the total energy to ~1e-8 where the network's own errors drift it
        # by ~1e-5 over the run; --long-time adds the run without it.  The
        # network learns from snapshots of a 1e7-particle beam: learned from
        # a 1e6-particle beam, whose field is noisier than that of the 1e8
        # evaluation beam, the same number of Adam steps left a 3x larger
        # median particle error at the end of the run
        line["learned_vs_plain_vp"] = compare.equal_error_vp(
            n_eval=args.learned_vp_eval, n_data=args.learned_vp_data,
            epochs=args.learned_vp_epochs,
            steps=args.learned_vp_steps, every=max(10, args.learned_vp_steps // 20),
            plain_Ks=(100, 200, 400), K_ref=1600, extra_tols=(), single_run=True, project=True,
            log=say)
        line["roofline_learned"] = learned_roofline(line)
    if not args.no_paper_schemes:
        from paper_1404_1160_amd import compare
        print("bench: the paper's self-consistent long run (eps 1e-3, t = 60)", file=sys.stderr,
              flush=True)
        runs = ((1e-3, 60.0, (10.0, 30.0, 60.0)),)
        if args.long_time:
            runs += ((1e-4, 90.0, (30.0, 60.0, 90.0)),)
        line["paper_schemes_long_vp"] = compare.paper_schemes_long_vp(
            runs=runs, log=lambda m: print("bench: " + m, file=sys.stderr, flush=True))
    if args.long_time and not args.no_learned:
        from paper_1404_1160_amd import compare
        print("bench: learned-vs-plain comparison, Vlasov-Poisson at scale, no projection",
              file=sys.stderr, flush=True)
        line["learned_vs_plain_vp_unprojected"] = compare.equal_error_vp(
            n_eval=args.learned_vp_eval, n_data=args.learned_vp_data,
            epochs=args.learned_vp_epochs,
            steps=args.learned_vp_steps, every=max(10, args.learned_vp_steps // 20),
            plain_Ks=(100, 200, 400), K_ref=1600, extra_tols=(), single_run=True, project=False,
            log=lambda m: print("bench: " + m, file=sys.stderr, flush=True))
    if args.long_time:
        from paper_1404_1160_amd import compare
        print("bench: long-time learned Vlasov-Poisson run", file=sys.stderr, flush=True)
        line["long_time_vp"] = compare.long_time_vp(
            log=lambda m: print("bench: " + m, file=sys.stderr, flush=True))
        print("bench: long-time Duffing run with the base-push network", file=sys.stderr,
              flush=True)
        line["long_time_duffing"] = compare.long_time_duffing(
            log=lambda m: print("bench: " + m, file=sys.stderr, flush=True))
        print("bench: the paper's schemes to t = 90", file=sys.stderr, flush=True)
        line["paper_schemes_long"] = compare.paper_schemes_long(
            log=lambda m: print("bench: " + m, file=sys.stderr, flush=True))
    if not args.no_paper_schemes:
        from paper_1404_1160_amd import compare
        print("bench: the paper's schemes (reference RK4, improved ETD)", file=sys.stderr,
              flush=True)
        line["paper_schemes"] = compare.paper_schemes(
            n_duffing=1_000_000, n_vp=100_000, steps_duffing=20, steps_vp=2,
            log=lambda m: print("bench: " + m, file=sys.stderr, flush=True))
        line["period_diagnostics"] = compare.period_diagnostics()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(n, args.cells, args.eps, args.dt, args.substeps,
                                            args.cpu_seconds)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
