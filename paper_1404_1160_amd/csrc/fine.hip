// Host side of the paper's own solvers: the reference RK4 solver, the
// improved ETD scheme (Algorithm 3.4) and the classic / modified ETD scheme
// (Algorithm 2.1), push modes EP_PUSH_RK4, EP_PUSH_IMPROVED_ETD,
// EP_PUSH_CLASSIC_ETD and EP_PUSH_MODIFIED_ETD of ep_step.

#include "context.h"

using namespace etd;

namespace {

constexpr long long kSearchChunk = 16;   // period-search steps between progress checks
constexpr int kRedBlocks = 256;          // partial sums of the mean-period reduction

ep_status ensure_fine(ep_ctx *c, bool coupled)
{
    FineArgs &a = c->fine;
    if (c->fine_cap >= c->n && a.T && (!coupled || a.yR)) return EP_OK;
    free_fine(c);
    const size_t n = (size_t)(c->n ? c->n : 1);
    HIPCHK(c, dalloc(&a.T, n));
    HIPCHK(c, dalloc(&a.N, n));
    HIPCHK(c, dalloc(&a.done, (size_t)3));
    a.last = a.done + 1;
    a.unresolved = a.done + 2;
    HIPCHK(c, dalloc(&a.red, (size_t)(kRedBlocks + 1)));
    if (coupled) {
        for (double **p : {&a.yR, &a.yV, &a.sR, &a.sV, &a.aR, &a.aV, &a.pR, &a.pV, &a.cR, &a.cV,
                           &a.dR, &a.dV, &a.t1, &a.o})
            HIPCHK(c, dalloc(p, n));
        HIPCHK(c, dalloc(&a.cnt, n));
    }
    c->fine_cap = c->n;
    return EP_OK;
}

uint64_t read_counter(ep_ctx *c, const unsigned long long *d, hipError_t &e)
{
    unsigned long long v = 0;
    e = hipMemcpyAsync(&v, d, sizeof v, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return v;
}

// Field of the start level (FP64 positions y) into the mesh.
ep_status start_field(ep_ctx *c, const MeshArgs &ma)
{
    HIPCHK(c, timed_launch(c, "fine_deposit", [&] {
               return launch_fine_deposit(c->stream, c->fine.yR, (int64_t)c->n, ma,
                                          c->push_grid_cap);
           }));
    return solve_mesh(c, ma, false);
}

// One coupled RK4 step to level L: four stages, each followed by a solve.
ep_status coupled_step(ep_ctx *c, int mode, double h, double eps, long long L, const MeshArgs &ma)
{
    for (int stage = 1; stage <= 4; ++stage) {
        HIPCHK(c, timed_launch(c, "fine_stage", [&] {
                   return launch_rk4_stage(c->stream, stage, mode, c->fine, (int64_t)c->n, h, eps,
                                           L, ma, c->push_grid_cap);
               }));
        if (ep_status s = solve_mesh(c, ma, false); s != EP_OK) return s;
    }
    return EP_OK;
}

// Period search in lock step from the state z at phase rot0: until every
// particle has its third sign change of V, or max_fine fine steps.
ep_status coupled_period_search(ep_ctx *c, double h, double eps, double2 rot0, const MeshArgs &ma)
{
    FineArgs &a = c->fine;
    const int64_t n = (int64_t)c->n;
    hipError_t e = hipSuccess;
    ep_status s;
    HIPCHK(c, hipMemsetAsync(a.done, 0, 3 * sizeof(unsigned long long), c->stream));
    HIPCHK(c, launch_fine_begin(c->stream, a, c->zR, c->zV, n, rot0, 1, eps));
    if ((s = start_field(c, ma)) != EP_OK) return s;
    long long L = 0;
    while (L < (long long)c->max_fine) {
        long long chunk = kSearchChunk;
        if (chunk > (long long)c->max_fine - L) chunk = (long long)c->max_fine - L;
        for (long long j = 0; j < chunk; ++j)
            if ((s = coupled_step(c, 1, h, eps, ++L, ma)) != EP_OK) return s;
        const uint64_t done = read_counter(c, a.done, e);
        if (e != hipSuccess) return c->hipfail("ep_step: period search", e);
        if (done >= c->n) break;
    }
    return EP_OK;
}

}  // namespace

namespace etd {

void free_fine(ep_ctx *c)
{
    FineArgs &a = c->fine;
    for (void *p : {(void *)a.yR, (void *)a.yV, (void *)a.sR, (void *)a.sV, (void *)a.aR,
                    (void *)a.aV, (void *)a.pR, (void *)a.pV, (void *)a.cR, (void *)a.cV,
                    (void *)a.dR, (void *)a.dV, (void *)a.t1, (void *)a.T, (void *)a.o,
                    (void *)a.cnt, (void *)a.N, (void *)a.done, (void *)a.red})
        if (p) (void)hipFree(p);
    a = FineArgs();
    c->fine_cap = 0;
    c->periods_valid = false;
}

ep_status fine_steps(ep_ctx *c, double dt, double eps, int32_t field, uint64_t n_steps)
{
    const bool ietd = c->push_mode == EP_PUSH_IMPROVED_ETD;
    const bool modified = c->push_mode == EP_PUSH_MODIFIED_ETD;
    const bool classic = modified || c->push_mode == EP_PUSH_CLASSIC_ETD;
    const bool coupled = field == EP_FIELD_POISSON;
    const double h = c->h_fine > 0.0 ? c->h_fine : kTwoPi * eps / 100.0;
    const double dphi = fmod(dt / eps, kTwoPi);
    ep_status s = ensure_fine(c, coupled);
    if (s != EP_OK) return s;
    const MeshArgs ma = c->mesh();
    const int64_t n = (int64_t)c->n;
    FineArgs &a = c->fine;
    hipError_t e = hipSuccess;
    for (uint64_t step = 0; step < n_steps; ++step) {
        const double p0 = c->phase, p1 = fmod(c->phase + dphi, kTwoPi);
        const double2 rot0 = make_double2(cos(p0), sin(p0)), rot1 = make_double2(cos(p1), sin(p1));
        if (classic) {
            // Algorithm 2.1 with P = 2 pi eps, or with the mean period
            double P = kTwoPi * eps;
            if (modified) {
                HIPCHK(c, hipMemsetAsync(a.done, 0, 3 * sizeof(unsigned long long), c->stream));
                if (!coupled) {
                    HIPCHK(c, timed_launch(c, "period_duffing", [&] {
                               return launch_period_duffing(c->stream, c->zR, c->zV, n, h, eps,
                                                            (long long)c->max_fine, rot0, a.T,
                                                            a.unresolved);
                           }));
                } else {
                    if ((s = coupled_period_search(c, h, eps, rot0, ma)) != EP_OK) return s;
                    HIPCHK(c, launch_ietd_split(c->stream, a, n, dt, h));   // counts unresolved
                }
                HIPCHK(c, launch_sum(c->stream, a.T, n, a.red, kRedBlocks, a.red + kRedBlocks));
                double sum = 0.0;
                HIPCHK(c, hipMemcpyAsync(&sum, a.red + kRedBlocks, sizeof sum,
                                         hipMemcpyDeviceToHost, c->stream));
                HIPCHK(c, hipStreamSynchronize(c->stream));
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
            long long K1 = (long long)ceil(P / h - 1e-9);
            if (K1 < 1) K1 = 1;
            long long K2 = o > 0.0 ? (long long)ceil(o / h - 1e-9) : 0;
            if (o > 0.0 && K2 < 1) K2 = 1;
            const double hP = P / (double)K1, ho = K2 ? o / (double)K2 : 0.0;
            if (!coupled) {
                HIPCHK(c, timed_launch(c, "cetd_duffing", [&] {
                           return launch_cetd_duffing(c->stream, c->zR, c->zV, n, hP, K1, ho, K2,
                                                      q, eps, rot0, rot1);
                       }));
            } else {
                HIPCHK(c, launch_fine_begin(c->stream, a, c->zR, c->zV, n, rot0, 3, eps));
                if ((s = start_field(c, ma)) != EP_OK) return s;
                for (long long L = 1; L <= K1; ++L)
                    if ((s = coupled_step(c, 0, hP, eps, L, ma)) != EP_OK) return s;
                HIPCHK(c, launch_cetd_combine(c->stream, a, n, q));
                if ((s = start_field(c, ma)) != EP_OK) return s;
                for (long long L = 1; L <= K2; ++L)
                    if ((s = coupled_step(c, 0, ho, eps, L, ma)) != EP_OK) return s;
                HIPCHK(c, launch_fine_end(c->stream, a, c->zR, c->zV, n, rot1, 0));
            }
            if (modified) HIPCHK(c, launch_fill_ll(c->stream, a.N, n, (long long)q));
            c->last_period = P;
        } else if (!ietd) {
            long long K = (long long)ceil(dt / h - 1e-9);
            if (K < 1) K = 1;
            const double hk = dt / (double)K;
            if (!coupled) {
                HIPCHK(c, timed_launch(c, "rk4_duffing", [&] {
                           return launch_rk4_duffing(c->stream, c->zR, c->zV, n, hk, eps, K, rot0,
                                                     rot1);
                       }));
            } else {
                HIPCHK(c, launch_fine_begin(c->stream, a, c->zR, c->zV, n, rot0, 0, eps));
                if ((s = start_field(c, ma)) != EP_OK) return s;
                for (long long L = 1; L <= K; ++L)
                    if ((s = coupled_step(c, 0, hk, eps, L, ma)) != EP_OK) return s;
                HIPCHK(c, launch_fine_end(c->stream, a, c->zR, c->zV, n, rot1, 0));
            }
        } else if (!coupled) {
            // the periods of an earlier search stay valid in the given field;
            // the unresolved count stays that of the search
            const bool reuse = c->periods_once && c->periods_valid && c->periods_duffing &&
                               c->periods_eps == eps && c->periods_h == h &&
                               c->periods_step == c->n_steps;
            if (!reuse)
                HIPCHK(c, hipMemsetAsync(a.unresolved, 0, sizeof(unsigned long long), c->stream));
            HIPCHK(c, timed_launch(c, reuse ? "ietd_duffing_reuse" : "ietd_duffing", [&] {
                       return launch_ietd_duffing(c->stream, c->zR, c->zV, n, dt, h, eps,
                                                  (long long)c->max_fine, rot0, rot1, reuse, a.T,
                                                  a.N, a.unresolved);
                   }));
        } else if (ietd) {
            // (a) period search, all particles in lock step until every one
            // has its third sign change of V (or max_fine steps)
            if ((s = coupled_period_search(c, h, eps, rot0, ma)) != EP_OK) return s;
            // (b) dt = N T + o, and the last fine level the captures need
            HIPCHK(c, launch_ietd_split(c->stream, a, n, dt, h));
            const uint64_t last = read_counter(c, a.last, e);
            if (e != hipSuccess) return c->hipfail("ep_step: split", e);
            // (c) second solve from y^n with the captures, (d) combination
            HIPCHK(c, launch_fine_begin(c->stream, a, c->zR, c->zV, n, rot0, 2, eps));
            if ((s = start_field(c, ma)) != EP_OK) return s;
            for (long long Lc = 1; Lc <= (long long)last; ++Lc)
                if ((s = coupled_step(c, 2, h, eps, Lc, ma)) != EP_OK) return s;
            HIPCHK(c, launch_fine_end(c->stream, a, c->zR, c->zV, n, rot1, 1));
        }
        c->phase = p1;
        c->t += dt;
        c->n_steps += 1;
        c->periods_valid = ietd || modified;
        c->periods_duffing = (ietd || modified) && !coupled;
        c->periods_eps = eps;
        c->periods_h = h;
        c->periods_step = c->n_steps;
    }
    c->field_valid = false;
    return EP_OK;
}

ep_status restore_periods(ep_ctx *c, const double *T, const int64_t *N, uint64_t unresolved)
{
    ep_status s = ensure_fine(c, false);
    if (s != EP_OK) return s;
    FineArgs &a = c->fine;
    const unsigned long long un = unresolved;
    if (c->n) {
        HIPCHK(c, copy_sync(c, a.T, T, c->n * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(c, copy_sync(c, a.N, N, c->n * sizeof(int64_t), hipMemcpyHostToDevice));
    }
    HIPCHK(c, copy_sync(c, a.unresolved, &un, sizeof un, hipMemcpyHostToDevice));
    return EP_OK;
}

}  // namespace etd

extern "C" {

ep_status ep_set_fine_solver(ep_ctx *c, double h_fine, uint64_t max_fine, int32_t periods_once)
{
    if (!c) return EP_EINVAL;
    if (!(h_fine == h_fine) || !isfinite(h_fine) || max_fine == 0)
        return c->fail(EP_EINVAL, "ep_set_fine_solver: need a finite h_fine and max_fine >= 1");
    if (periods_once != 0 && periods_once != 1)
        return c->fail(EP_EINVAL, "ep_set_fine_solver: periods_once must be 0 or 1");
    c->h_fine = h_fine;
    c->max_fine = max_fine;
    c->periods_once = periods_once != 0;
    c->periods_duffing = false;   // a new max_fine may resolve other periods
    return EP_OK;
}

ep_status ep_compute_periods(ep_ctx *c, double eps, int32_t field, uint64_t *n_unresolved)
{
    if (!c) return EP_EINVAL;
    if (!(eps > 0.0) || !isfinite(eps) || (field != EP_FIELD_DUFFING && field != EP_FIELD_POISSON))
        return c->fail(EP_EINVAL, "ep_compute_periods: need eps > 0 and the Duffing or Poisson "
                                  "field");
    if (c->w <= 0.0) return c->fail(EP_ESTATE, "ep_compute_periods: no particles loaded");
    if (c->cfg.deposit == EP_DEPOSIT_SORTED)
        return c->fail(EP_EINVAL, "ep_compute_periods: not with the sorted deposit");
    DeviceGuard guard(c->device);
    const bool coupled = field == EP_FIELD_POISSON;
    ep_status s = ensure_fine(c, coupled);
    if (s != EP_OK) return s;
    FineArgs &a = c->fine;
    const int64_t n = (int64_t)c->n;
    const double h = c->h_fine > 0.0 ? c->h_fine : kTwoPi * eps / 100.0;
    const double2 rot0 = make_double2(cos(c->phase), sin(c->phase));
    HIPCHK(c, hipMemsetAsync(a.done, 0, 3 * sizeof(unsigned long long), c->stream));
    if (!coupled) {
        HIPCHK(c, launch_period_duffing(c->stream, c->zR, c->zV, n, h, eps, (long long)c->max_fine,
                                        rot0, a.T, a.unresolved));
    } else {
        if ((s = coupled_period_search(c, h, eps, rot0, c->mesh())) != EP_OK) return s;
        HIPCHK(c, launch_ietd_split(c->stream, a, n, 0.0, h));   // counts unresolved
        c->field_valid = false;
    }
    HIPCHK(c, launch_fill_ll(c->stream, a.N, n, 0));
    unsigned long long un = 0;
    HIPCHK(c, hipMemcpyAsync(&un, a.unresolved, sizeof un, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->periods_valid = true;
    c->periods_duffing = !coupled;
    c->periods_eps = eps;
    c->periods_h = h;
    c->periods_step = c->n_steps;
    if (n_unresolved) *n_unresolved = un;
    return EP_OK;
}

ep_status ep_get_periods(ep_ctx *c, double *T, int64_t *N, uint64_t offset, uint64_t count,
                         uint64_t *n_unresolved)
{
    if (!c) return EP_EINVAL;
    if (!c->periods_valid)
        return c->fail(EP_ESTATE, "ep_get_periods: no improved-ETD step since the particles "
                                  "were set");
    if (offset > c->n || count > c->n - offset)
        return c->fail(EP_EINVAL, "ep_get_periods: range outside the %llu particles",
                       (unsigned long long)c->n);
    DeviceGuard guard(c->device);
    if (count && T)
        HIPCHK(c, hipMemcpyAsync(T, c->fine.T + offset, count * sizeof(double),
                                 hipMemcpyDeviceToHost, c->stream));
    if (count && N)
        HIPCHK(c, hipMemcpyAsync(N, c->fine.N + offset, count * sizeof(int64_t),
                                 hipMemcpyDeviceToHost, c->stream));
    unsigned long long un = 0;
    HIPCHK(c, hipMemcpyAsync(&un, c->fine.unresolved, sizeof un, hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (n_unresolved) *n_unresolved = un;
    return EP_OK;
}

}  // extern "C"
