/*
 * Plain FP64 CPU oracle of the paper's own solvers.
 *
 * TEST INFRASTRUCTURE ONLY, like pic_oracle.c (built into the same library,
 * loaded only by the tests, the smoke check and the benchmark's CPU leg).
 *
 * 1. Reference solver: the classic fourth-order Runge-Kutta method on the
 *    characteristics of eq. 1.4, y' = (1/eps) M y + (0, E(t, R)), with a
 *    small step (the paper uses 2 pi eps / 100, section 2).  For the
 *    self-consistent field the charge of all particles is deposited and the
 *    Poisson equation (eq. 1.2) solved again at every stage, from the stage
 *    positions, so the particles advance together.
 *
 * 2. The improved ETD scheme (Algorithm 3.4), one macro step dt:
 *    (a) periods T_i: each particle is solved with the reference solver
 *        until its velocity has changed sign three times; the period is the
 *        time between the first and the third sign change (Remark 3.5);
 *    (b) dt = N_i T_i + o_i with N_i a whole number and 0 <= o_i < T_i;
 *    (c) y_i(t_n + o_i) and y_i(t_n + o_i + T_i) from a second reference
 *        solve started at y_i^n, by quadratic interpolation on the fine
 *        grid (Remark 3.6);
 *    (d) y_i^{n+1} = y_i(t_n + o_i) + N_i (y_i(t_n + o_i + T_i) - y_i(t_n + o_i))
 *        (Lemma 3.3).
 *
 * 3. The classic ETD scheme (Algorithm 2.1) with a common fast period P, and
 *    its modified form, P = the mean over the particles of their periods T_i
 *    (section 2): dt = N P + o; a reference solve over P from y^n gives
 *    y(t_n + P); y(t_n + N P) = y^n + N (y(t_n + P) - y^n) (its step 2); a
 *    reference solve over o from there gives y^{n+1}.  The solves over P and
 *    o take ceil(P / h) and ceil(o / h) equal steps (at least one for o > 0).
 *
 * Readings where the paper is silent:
 *   - a sign change of V between fine levels k and k+1 is (V_k < 0) !=
 *     (V_{k+1} < 0); its time is found by linear interpolation of V between
 *     the two levels (V is close to linear there: R has an extremum);
 *   - the quadratic interpolation for a time tau uses the fine levels j-1,
 *     j, j+1 around the level j nearest to tau (j >= 1);
 *   - a particle whose velocity has not changed sign three times after
 *     max_fine fine steps keeps the free period 2 pi eps (it is counted).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { F_ZERO = 0, F_DUFFING = 1, F_POISSON = 2, F_CONST = 3 };

/* from pic_oracle.c (same library) */
int64_t orc_deposit(const double *R, int64_t n, double w, int nr, double rmin, double rmax,
                    double *rho);
void orc_poisson(const double *rho, int nr, double rmin, double rmax, double *E, double *Psi,
                 double *Qb);
double orc_gather(double R, const double *E, double Qb, int nr, double rmin, double rmax);

typedef struct {
    int kind;
    double E0, w;
    int nr;
    double rmin, rmax;
    double *rho, *E;
    double Qb;
} field_ctx;

/* The field of the current stage: for the Poisson field, deposit the stage
 * positions of all particles and solve. */
static void field_prepare(field_ctx *f, const double *R, int64_t n)
{
    if (f->kind != F_POISSON) return;
    orc_deposit(R, n, f->w, f->nr, f->rmin, f->rmax, f->rho);
    orc_poisson(f->rho, f->nr, f->rmin, f->rmax, f->E, NULL, &f->Qb);
}

static double field_eval(const field_ctx *f, double R)
{
    switch (f->kind) {
    case F_DUFFING: return -R * R * R;
    case F_POISSON: return orc_gather(R, f->E, f->Qb, f->nr, f->rmin, f->rmax);
    case F_CONST: return f->E0;
    default: return 0.0;
    }
}

/* One classic RK4 step of size h for all particles (coupled through the field).
 * work: 6n doubles. */
static void rk4_step(double *R, double *V, int64_t n, double eps, double h, field_ctx *f,
                     double *work)
{
    double *sR = work, *sV = work + n, *aR = work + 2 * n, *aV = work + 3 * n;
    (void)aV;
    const double ie = 1.0 / eps;
    /* k1 at y */
    field_prepare(f, R, n);
    for (int64_t i = 0; i < n; ++i) {
        const double kR = V[i] * ie, kV = -R[i] * ie + field_eval(f, R[i]);
        aR[i] = kR;
        aV[i] = kV;
        sR[i] = R[i] + 0.5 * h * kR;
        sV[i] = V[i] + 0.5 * h * kV;
    }
    /* k2 at y + h/2 k1, k3 at y + h/2 k2 */
    for (int stage = 2; stage <= 3; ++stage) {
        field_prepare(f, sR, n);
        const double c = stage == 2 ? 0.5 * h : h;
        for (int64_t i = 0; i < n; ++i) {
            const double kR = sV[i] * ie, kV = -sR[i] * ie + field_eval(f, sR[i]);
            aR[i] += 2.0 * kR;
            aV[i] += 2.0 * kV;
            sR[i] = R[i] + c * kR;
            sV[i] = V[i] + c * kV;
        }
    }
    /* k4 at y + h k3 */
    field_prepare(f, sR, n);
    for (int64_t i = 0; i < n; ++i) {
        const double kR = sV[i] * ie, kV = -sR[i] * ie + field_eval(f, sR[i]);
        R[i] += h / 6.0 * (aR[i] + kR);
        V[i] += h / 6.0 * (aV[i] + kV);
    }
}

static int field_init(field_ctx *f, int kind, double E0, double w, int nr, double rmin,
                      double rmax)
{
    memset(f, 0, sizeof *f);
    f->kind = kind;
    f->E0 = E0;
    f->w = w;
    f->nr = nr;
    f->rmin = rmin;
    f->rmax = rmax;
    if (kind == F_POISSON) {
        f->rho = (double *)malloc(sizeof(double) * (size_t)(nr + 1));
        f->E = (double *)malloc(sizeof(double) * (size_t)(nr + 1));
        if (!f->rho || !f->E) return -1;
    }
    return 0;
}

static void field_free(field_ctx *f)
{
    free(f->rho);
    free(f->E);
}

/* n_steps reference steps of size h. Returns 0, or -1 without memory. */
int orc_rk4_run(double *R, double *V, int64_t n, double w, double eps, double h, int64_t n_steps,
                int kind, double E0, int nr, double rmin, double rmax)
{
    field_ctx f;
    double *work = (double *)malloc(sizeof(double) * (size_t)(6 * (n > 0 ? n : 1)));
    if (!work || field_init(&f, kind, E0, w, nr, rmin, rmax) != 0) {
        free(work);
        return -1;
    }
    for (int64_t s = 0; s < n_steps; ++s) rk4_step(R, V, n, eps, h, &f, work);
    field_free(&f);
    free(work);
    return 0;
}

/* Quadratic interpolation at u = (tau - t_j)/h through levels j-1, j, j+1. */
static double quad(double a, double b, double c, double u)
{
    return a * (0.5 * u * (u - 1.0)) + b * (1.0 - u * u) + c * (0.5 * u * (u + 1.0));
}

/* Nearest fine level to tau, at least 1. */
static int64_t near_level(double tau, double h)
{
    int64_t j = (int64_t)floor(tau / h + 0.5);
    return j < 1 ? 1 : j;
}

/* Period search: the reference solve from (R, V) until every particle's
 * velocity has changed sign three times or max_fine steps; T[i] receives the
 * time from the first to the third change (2 pi eps if not found).  Returns
 * the number of unresolved particles.  buf: 3n doubles, cnt: n ints (zeroed
 * here), work: 6n doubles. */
static int64_t period_search(const double *R, const double *V, int64_t n, double eps, double h,
                             field_ctx *f, int64_t max_fine, double *T, double *buf, int *cnt,
                             double *work)
{
    const size_t nn = (size_t)n;
    double *Rw = buf, *Vw = buf + nn, *t1 = buf + 2 * nn;
    double *Vp = work + 4 * nn;   /* the part of work rk4_step leaves alone */
    memcpy(Rw, R, sizeof(double) * nn);
    memcpy(Vw, V, sizeof(double) * nn);
    memset(cnt, 0, sizeof(int) * nn);
    for (int64_t i = 0; i < n; ++i) T[i] = 2.0 * M_PI * eps;
    int64_t done = 0, steps = 0;
    while (done < n && steps < max_fine) {
        memcpy(Vp, Vw, sizeof(double) * nn);
        rk4_step(Rw, Vw, n, eps, h, f, work);
        for (int64_t i = 0; i < n; ++i) {
            if (cnt[i] >= 3 || (Vp[i] < 0.0) == (Vw[i] < 0.0)) continue;
            const double ts = (double)steps * h + h * Vp[i] / (Vp[i] - Vw[i]);
            cnt[i] += 1;
            if (cnt[i] == 1) t1[i] = ts;
            if (cnt[i] == 3) {
                T[i] = ts - t1[i];
                ++done;
            }
        }
        ++steps;
    }
    return n - done;
}

/* Reference solve over a duration d in ceil(d / h) equal steps. */
static void solve_for(double *R, double *V, int64_t n, double eps, double d, double h,
                      field_ctx *f, double *work)
{
    if (!(d > 0.0)) return;
    int64_t K = (int64_t)ceil(d / h - 1e-9);
    if (K < 1) K = 1;
    const double hk = d / (double)K;
    for (int64_t k = 0; k < K; ++k) rk4_step(R, V, n, eps, hk, f, work);
}

/* One macro step of the classic ETD scheme (Algorithm 2.1) with the period
 * 2 pi eps (modified = 0) or with the mean period of the particles
 * (modified = 1; T receives the periods).  *P_out receives the period used.
 * Returns the number of unresolved particles (modified), or -1 without
 * memory. */
int64_t orc_classic_etd_step(double *R, double *V, int64_t n, double w, double dt, double eps,
                             double h, int kind, double E0, int nr, double rmin, double rmax,
                             int modified, int64_t max_fine, double *T, double *P_out)
{
    if (n <= 0) return 0;
    field_ctx f;
    const size_t nn = (size_t)n;
    double *work = (double *)malloc(sizeof(double) * 6 * nn);
    double *buf = (double *)malloc(sizeof(double) * 5 * nn);
    int *cnt = (int *)calloc(nn, sizeof(int));
    if (!work || !buf || !cnt || field_init(&f, kind, E0, w, nr, rmin, rmax) != 0) {
        free(work);
        free(buf);
        free(cnt);
        return -1;
    }
    double P = 2.0 * M_PI * eps;
    int64_t unresolved = 0;
    if (modified) {
        unresolved = period_search(R, V, n, eps, h, &f, max_fine, T, buf, cnt, work);
        double sum = 0.0;
        for (int64_t i = 0; i < n; ++i) sum += T[i];
        P = sum / (double)n;
    }
    double q = floor(dt / P), o = dt - q * P;
    if (o < 0.0) {
        q -= 1.0;
        o += P;
    }
    if (o >= P) {
        q += 1.0;
        o -= P;
    }
    double *Rp = buf + 3 * nn, *Vp = buf + 4 * nn;
    memcpy(Rp, R, sizeof(double) * nn);
    memcpy(Vp, V, sizeof(double) * nn);
    solve_for(Rp, Vp, n, eps, P, h, &f, work);                 /* y(t_n + P)   */
    for (int64_t i = 0; i < n; ++i) {                           /* y(t_n + N P) */
        R[i] = R[i] + q * (Rp[i] - R[i]);
        V[i] = V[i] + q * (Vp[i] - V[i]);
    }
    solve_for(R, V, n, eps, o, h, &f, work);                    /* y(t_{n+1})   */
    if (P_out) *P_out = P;
    field_free(&f);
    free(work);
    free(buf);
    free(cnt);
    return unresolved;
}

/* One macro step of the improved ETD scheme (Algorithm 3.4).  On return R, V
 * hold y^{n+1}; T[i] the period and N[i] the whole number of periods used.
 * Returns the number of particles whose period was not resolved within
 * max_fine fine steps (they use 2 pi eps), or -1 without memory.
 * alt_window > 0: a particle whose dt / T_i lies within alt_window of a whole
 * number m takes the other of the two splits dt = N T_i + o_i that hold there
 * up to rounding (N = m with o_i near 0, or N = m - 1 with o_i near T_i), with
 * o_i = dt - N T_i; the default split is the one with 0 <= o_i < T_i. */
int64_t orc_improved_etd_step(double *R, double *V, int64_t n, double w, double dt, double eps,
                              double h, int kind, double E0, int nr, double rmin, double rmax,
                              int64_t max_fine, int periods_given, double *T, int64_t *N,
                              double alt_window)
{
    if (n <= 0) return 0;
    field_ctx f;
    const size_t nn = (size_t)n;
    double *work = (double *)malloc(sizeof(double) * 6 * nn);
    double *buf = (double *)malloc(sizeof(double) * 16 * nn);
    int *cnt = (int *)calloc(nn, sizeof(int));
    if (!work || !buf || !cnt || field_init(&f, kind, E0, w, nr, rmin, rmax) != 0) {
        free(work);
        free(buf);
        free(cnt);
        return -1;
    }
    double *Rw = buf, *Vw = buf + nn, *Vp = buf + 2 * nn, *t1 = buf + 3 * nn, *o = buf + 4 * nn;
    double *Rl[3] = {buf + 5 * nn, buf + 6 * nn, buf + 7 * nn};
    double *Vl[3] = {buf + 8 * nn, buf + 9 * nn, buf + 10 * nn};
    double *Ra = buf + 11 * nn, *Va = buf + 12 * nn, *Rb = buf + 13 * nn, *Vb = buf + 14 * nn;
    double *ta = buf + 15 * nn;
    const double two_pi_eps = 2.0 * M_PI * eps;

    /* (a) periods; skipped when T holds them already (the given field keeps
       each particle's period constant, so the paper computes them at the
       first macro step only) */
    memcpy(Rw, R, sizeof(double) * nn);
    memcpy(Vw, V, sizeof(double) * nn);
    int64_t done = periods_given ? n : 0, steps = 0;
    if (!periods_given)
        for (int64_t i = 0; i < n; ++i) T[i] = two_pi_eps;
    while (done < n && steps < max_fine) {
        memcpy(Vp, Vw, sizeof(double) * nn);
        rk4_step(Rw, Vw, n, eps, h, &f, work);
        for (int64_t i = 0; i < n; ++i) {
            if (cnt[i] >= 3 || (Vp[i] < 0.0) == (Vw[i] < 0.0)) continue;
            const double ts = (double)steps * h + h * Vp[i] / (Vp[i] - Vw[i]);
            cnt[i] += 1;
            if (cnt[i] == 1) t1[i] = ts;
            if (cnt[i] == 3) {
                T[i] = ts - t1[i];
                ++done;
            }
        }
        ++steps;
    }
    const int64_t unresolved = n - done;

    /* (b) dt = N T + o */
    int64_t last = 0;
    for (int64_t i = 0; i < n; ++i) {
        double q = floor(dt / T[i]);
        double oi = dt - q * T[i];
        if (oi < 0.0) {
            q -= 1.0;
            oi += T[i];
        }
        if (oi >= T[i]) {
            q += 1.0;
            oi -= T[i];
        }
        if (alt_window > 0.0) {
            const double x = dt / T[i], m = floor(x + 0.5);
            if (fabs(x - m) <= alt_window) {
                q = q == m ? m - 1.0 : m;
                oi = dt - q * T[i];
            }
        }
        N[i] = (int64_t)q;
        o[i] = oi;
        ta[i] = oi + T[i];
        const int64_t lb = near_level(ta[i], h) + 1;
        if (lb > last) last = lb;
    }

    /* (c) second reference solve from y^n; level L is kept in slot L % 3 */
    memcpy(Rl[0], R, sizeof(double) * nn);
    memcpy(Vl[0], V, sizeof(double) * nn);
    memcpy(Rw, R, sizeof(double) * nn);
    memcpy(Vw, V, sizeof(double) * nn);
    for (int64_t L = 1; L <= last; ++L) {
        rk4_step(Rw, Vw, n, eps, h, &f, work);
        memcpy(Rl[L % 3], Rw, sizeof(double) * nn);
        memcpy(Vl[L % 3], Vw, sizeof(double) * nn);
        if (L < 2) continue;
        const int a0 = (int)((L - 2) % 3), a1 = (int)((L - 1) % 3), a2 = (int)(L % 3);
        for (int64_t i = 0; i < n; ++i) {
            const double tau[2] = {o[i], ta[i]};
            double *outR[2] = {Ra, Rb}, *outV[2] = {Va, Vb};
            for (int m = 0; m < 2; ++m) {
                const int64_t j = near_level(tau[m], h);
                if (j + 1 != L) continue;
                const double u = (tau[m] - (double)j * h) / h;
                outR[m][i] = quad(Rl[a0][i], Rl[a1][i], Rl[a2][i], u);
                outV[m][i] = quad(Vl[a0][i], Vl[a1][i], Vl[a2][i], u);
            }
        }
    }

    /* (d) extrapolation over N whole periods */
    for (int64_t i = 0; i < n; ++i) {
        const double q = (double)N[i];
        R[i] = Ra[i] + q * (Rb[i] - Ra[i]);
        V[i] = Va[i] + q * (Vb[i] - Va[i]);
    }
    field_free(&f);
    free(work);
    free(buf);
    free(cnt);
    return unresolved;
}
