/* etdpic_run: a command-line driver of the PIC step through the C ABI.
 *
 * It loads a Gaussian beam (R ~ N(0,1) truncated to |R| < 4, V ~ N(0,1),
 * equal weights), takes W untimed steps and S timed steps of the
 * self-consistent (Vlasov-Poisson) field, or of the Duffing field E = -R^3
 * (--field duffing; then R, V ~ N(0, 1.5) untruncated), at the given dt and
 * eps, and prints the step time; with --copy-bytes it also times a
 * device-to-device copy of that many bytes.  --deposit sorted selects the
 * sort-by-cell deposit.  With --learned bf16|fp16 the
 * steps are the learned push with a network of seeded Glorot-uniform weights
 * (5 or 6 inputs -> 64 -> 64 -> 2; its predictions are meaningless, its cost
 * is that of any network of this shape), the drift bound --drift-tol
 * (default: none, every particle takes the network's map) and K_fb =
 * --fallback-substeps; --base-substeps K_B (Duffing field) gives the network
 * a base push of K_B plain substeps.  One process, one HIP runtime and no Python, so a
 * hardware-counter profiler can wrap it directly.
 *
 * Usage: etdpic_run [--particles N] [--cells M] [--substeps K] [--steps S]
 *                   [--warmup W] [--dt DT] [--eps EPS] [--seed SEED]
 *                   [--field poisson|duffing] [--learned bf16|fp16]
 *                   [--drift-tol TOL] [--fallback-substeps K_FB] [--base-substeps K_B]
 *                   [--deposit atomic|sorted] [--copy-bytes B] [--copy-reps R]
 *
 * Exit status 0 on success, 1 on a bad argument or a library error (its
 * message goes to stderr).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#include "etdpic.h"

static uint64_t splitmix64(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* uniform in (0, 1] from the top 53 bits */
static double uniform01(uint64_t *s)
{
    return ((double)(splitmix64(s) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
}

/* two independent standard normals (Box-Muller) */
static void normal_pair(uint64_t *s, double *a, double *b)
{
    const double r = sqrt(-2.0 * log(uniform01(s)));
    const double phi = 6.283185307179586 * uniform01(s);
    *a = r * cos(phi);
    *b = r * sin(phi);
}

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static int check(ep_ctx *ctx, ep_status st, const char *what)
{
    if (st == EP_OK) return 0;
    fprintf(stderr, "etdpic_run: %s failed (%d): %s\n", what, (int)st,
            ctx ? ep_last_error(ctx) : "");
    return 1;
}

/* Seeded Glorot-uniform parameters of the n_in -> 64 -> 64 -> 2 network
 * (layout of ep_mlp_set_weights), biases zero. */
static float *network(int n_in, uint64_t seed, uint32_t *n_params)
{
    const int h = 64, out = 2;
    const uint32_t np = (uint32_t)(h * n_in + h + h * h + h + out * h + out);
    float *p = calloc(np, sizeof(float));
    if (!p) return NULL;
    uint64_t s = seed;
    const int fan[3][2] = {{n_in, h}, {h, h}, {h, out}};
    uint32_t at = 0;
    for (int l = 0; l < 3; ++l) {
        const double lim = sqrt(6.0 / (double)(fan[l][0] + fan[l][1]));
        for (int i = 0; i < fan[l][0] * fan[l][1]; ++i)
            p[at++] = (float)(lim * (2.0 * uniform01(&s) - 1.0));
        at += (uint32_t)fan[l][1];   /* biases */
    }
    *n_params = np;
    return p;
}

int main(int argc, char **argv)
{
    uint64_t n = 100000000ull, seed = 13, copy_bytes = 0;
    uint32_t cells = 4096, substeps = 1, fb_substeps = 400, base_substeps = 0;
    long steps = 20, warmup = 2, copy_reps = 10;
    double dt = 0.05, eps = 1e-3, drift_tol = 1e300;
    int field = EP_FIELD_POISSON, learned = -1, deposit = EP_DEPOSIT_ATOMIC;
    for (int i = 1; i < argc; ++i) {
        const char *a = argv[i];
        const char *v = i + 1 < argc ? argv[i + 1] : NULL;
        if (!v) {
            fprintf(stderr, "etdpic_run: %s needs a value\n", a);
            return 1;
        }
        if (!strcmp(a, "--particles")) n = strtoull(v, NULL, 10);
        else if (!strcmp(a, "--cells")) cells = (uint32_t)strtoul(v, NULL, 10);
        else if (!strcmp(a, "--substeps")) substeps = (uint32_t)strtoul(v, NULL, 10);
        else if (!strcmp(a, "--steps")) steps = strtol(v, NULL, 10);
        else if (!strcmp(a, "--warmup")) warmup = strtol(v, NULL, 10);
        else if (!strcmp(a, "--dt")) dt = strtod(v, NULL);
        else if (!strcmp(a, "--eps")) eps = strtod(v, NULL);
        else if (!strcmp(a, "--seed")) seed = strtoull(v, NULL, 10);
        else if (!strcmp(a, "--copy-bytes")) copy_bytes = strtoull(v, NULL, 10);
        else if (!strcmp(a, "--copy-reps")) copy_reps = strtol(v, NULL, 10);
        else if (!strcmp(a, "--drift-tol")) drift_tol = strtod(v, NULL);
        else if (!strcmp(a, "--fallback-substeps")) fb_substeps = (uint32_t)strtoul(v, NULL, 10);
        else if (!strcmp(a, "--base-substeps")) base_substeps = (uint32_t)strtoul(v, NULL, 10);
        else if (!strcmp(a, "--field") && !strcmp(v, "poisson")) field = EP_FIELD_POISSON;
        else if (!strcmp(a, "--field") && !strcmp(v, "duffing")) field = EP_FIELD_DUFFING;
        else if (!strcmp(a, "--learned") && !strcmp(v, "bf16")) learned = EP_MLP_BF16;
        else if (!strcmp(a, "--learned") && !strcmp(v, "fp16")) learned = EP_MLP_FP16;
        else if (!strcmp(a, "--deposit") && !strcmp(v, "atomic")) deposit = EP_DEPOSIT_ATOMIC;
        else if (!strcmp(a, "--deposit") && !strcmp(v, "sorted")) deposit = EP_DEPOSIT_SORTED;
        else {
            fprintf(stderr, "etdpic_run: unknown option %s\n", a);
            return 1;
        }
        ++i;
    }
    if (n == 0 || steps < 1 || warmup < 0 || copy_reps < 1) {
        fprintf(stderr, "etdpic_run: need particles >= 1, steps >= 1, warmup >= 0\n");
        return 1;
    }

    double *R = malloc(n * sizeof(double)), *V = malloc(n * sizeof(double));
    if (!R || !V) {
        fprintf(stderr, "etdpic_run: out of host memory for %llu particles\n",
                (unsigned long long)n);
        return 1;
    }
    uint64_t s = seed;
    for (uint64_t j = 0; j < n; ++j) {
        double r, v;
        if (field == EP_FIELD_DUFFING) {
            normal_pair(&s, &r, &v);
            R[j] = 1.5 * r;
            V[j] = 1.5 * v;
            continue;
        }
        do normal_pair(&s, &r, &v); while (fabs(r) >= 4.0);
        double v2, unused;
        normal_pair(&s, &v2, &unused);
        R[j] = r;
        V[j] = v2;
    }

    ep_config cfg;
    memset(&cfg, 0, sizeof cfg);
    cfg.n_particles = n;
    cfg.n_cells = cells;
    cfg.substeps = substeps;
    cfg.r_max = 5.0;
    cfg.deposit = deposit;
    cfg.device = 0;
    ep_ctx *ctx = NULL;
    if (check(NULL, ep_create(&cfg, &ctx), "ep_create")) return 1;
    int bad = check(ctx, ep_set_particles(ctx, R, V, n, 1.0 / (double)n), "ep_set_particles");
    free(R);
    free(V);
    if (!bad && learned >= 0) {
        const int n_in = field == EP_FIELD_POISSON ? 6 : 5;
        uint32_t np = 0;
        float *p = network(n_in, seed + 1, &np);
        /* s_in, s_t, s_E, mu_d, sig_d, mu_k, sig_k, output map, base push substeps */
        const double norm[9] = {field == EP_FIELD_POISSON ? 1.0 : 1.5, 100.0, 0.25, 0.05, 0.05,
                                0.0, 1e-3, field == EP_FIELD_POISSON ? 1.0 : 0.0,
                                (double)base_substeps};
        bad = !p || check(ctx, ep_mlp_set_weights(ctx, p, np, norm), "ep_mlp_set_weights");
        free(p);
        if (!bad) bad = check(ctx, ep_mlp_set_precision(ctx, learned), "ep_mlp_set_precision");
        if (!bad)
            bad = check(ctx, ep_set_push_mode(ctx, EP_PUSH_LEARNED, drift_tol, fb_substeps),
                        "ep_set_push_mode");
    }
    if (!bad && warmup > 0)
        bad = check(ctx, ep_step(ctx, dt, eps, field, (uint64_t)warmup), "ep_step");
    if (!bad) bad = check(ctx, ep_sync(ctx), "ep_sync");
    double t0 = now_s();
    if (!bad) bad = check(ctx, ep_step(ctx, dt, eps, field, (uint64_t)steps), "ep_step");
    if (!bad) bad = check(ctx, ep_sync(ctx), "ep_sync");
    const double t1 = now_s();
    ep_moments m;
    if (!bad) bad = check(ctx, ep_moments_get(ctx, eps, field, &m), "ep_moments_get");
    if (!bad) {
        const double ms = (t1 - t0) * 1e3 / (double)steps;
        printf("etdpic_run: %s%s, %llu particles, %u cells, K=%u, %ld steps: %.4f ms/step, "
               "%.4g particle-steps/s; rms radius %.9f, energy %.9g, fallbacks %llu\n",
               field == EP_FIELD_POISSON ? "poisson" : "duffing",
               learned < 0 ? "" : learned == EP_MLP_BF16 ? ", learned bf16" : ", learned fp16",
               (unsigned long long)n, cells, substeps, steps, ms, (double)n / (ms * 1e-3),
               m.rms_radius, m.energy, (unsigned long long)m.n_fallback);
        fflush(stdout);
    }
    ep_destroy(ctx);
    if (bad) return 1;
    if (copy_bytes) {
        double gbs = 0.0;
        if (check(NULL, ep_copy_bandwidth(0, copy_bytes, (int32_t)copy_reps, &gbs),
                  "ep_copy_bandwidth"))
            return 1;
        printf("etdpic_run: device copy of %llu bytes x %ld: %.1f GB/s (read + write)\n",
               (unsigned long long)copy_bytes, copy_reps, gbs);
    }
    return 0;
}
