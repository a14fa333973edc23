// Host runtime of the exponential-integrator PIC library: context, device
// buffers, FP64 phase bookkeeping, step scheduling and the C ABI of etdpic.h.

#include <mutex>

#include "context.h"

using namespace etd;

namespace {

std::string g_create_error;

void free_all(ep_ctx *c)
{
    for (void *p : {(void *)c->own_zR, (void *)c->own_zV, (void *)c->hist,
                    (void *)c->etab, (void *)c->rho64, (void *)c->E64, (void *)c->Psi64,
                    (void *)c->fscal, (void *)c->tab.sub, (void *)c->tab.endrot,
                    (void *)c->stageR, (void *)c->stageV, (void *)c->mpartial, (void *)c->mout,
                    (void *)c->rec[0], (void *)c->rec[1], (void *)c->ids, (void *)c->inv,
                    (void *)c->counts, (void *)c->total, (void *)c->starts, (void *)c->sums,
                    (void *)c->mcount, (void *)c->mout_count})
        if (p) (void)hipFree(p);
    for (auto &p : c->pending) c->event_pool.push_back(p.second);
    for (auto &ev : c->event_pool) {
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    free_learned(c);
    free_fine(c);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

}  // namespace

namespace etd {

void set_context_free_error(const char *msg) { g_create_error = msg; }

hipError_t raise_dynamic_lds(const void *kernel, int bytes)
{
    static std::mutex mu;
    static std::map<const void *, int> limit;
    std::lock_guard<std::mutex> lock(mu);
    int &cur = limit[kernel];
    if (bytes <= cur) return hipSuccess;
    const hipError_t e =
        hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess) cur = bytes;
    return e;
}

LaunchEvents &next_launch_events()
{
    static thread_local LaunchEvents ev;
    return ev;
}

hipError_t collect_timing(ep_ctx *c)
{
    if (c->pending.empty()) return hipSuccess;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return e;
    for (auto &p : c->pending) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, p.second.first, p.second.second);
        if (e != hipSuccess) return e;
        auto &acc = c->timed[p.first];
        acc.first += ms;
        acc.second += 1;
        c->event_pool.push_back(p.second);
    }
    c->pending.clear();
    return hipSuccess;
}

ep_status ensure_tables(ep_ctx *c, size_t entries, size_t steps)
{
    if (entries <= c->tab_cap && steps <= c->tab_cap) return EP_OK;
    size_t cap = entries > steps ? entries : steps;
    if (cap < 1024) cap = 1024;
    if (c->tab.sub) (void)hipFree(c->tab.sub);
    if (c->tab.endrot) (void)hipFree(c->tab.endrot);
    c->tab.sub = nullptr;
    c->tab.endrot = nullptr;
    c->tab_cap = 0;
    HIPCHK(c, dalloc(&c->tab.sub, cap));
    HIPCHK(c, dalloc(&c->tab.endrot, cap));
    c->tab_cap = cap;
    return EP_OK;
}

// Deposit the current state and solve for its field.
ep_status refresh_field(ep_ctx *c)
{
    const double2 er = make_double2(cos(c->phase), sin(c->phase));
    const MeshArgs ma = c->mesh();
    HIPCHK(c, timed_launch(c, "deposit", [&] {
               return launch_push_poisson(c->stream, false, c->zR, c->zV, (int64_t)c->n,
                                          nullptr, nullptr, er, 0, ma, c->push_grid_cap);
           }));
    ep_status s = solve_mesh(c, ma, true);
    if (s != EP_OK) return s;
    c->field_valid = true;
    return EP_OK;
}

ep_status solve_mesh(ep_ctx *c, const MeshArgs &ma, bool potential)
{
    HIPCHK(c, timed_launch(c, "mesh_solve",
                           [&] { return launch_mesh_solve(c->stream, ma, potential); }));
    c->potential_valid = potential;
    return EP_OK;
}

ep_status ensure_potential(ep_ctx *c)
{
    if (c->potential_valid) return EP_OK;
    HIPCHK(c, timed_launch(c, "potential", [&] { return launch_potential(c->stream, c->mesh()); }));
    c->potential_valid = true;
    return EP_OK;
}

// One Poisson step with the sorted deposit: count, offsets, scatter into the
// record buffer `out` (which becomes the state), segmented reduction, solve.
// The state before the step is record buffer `in`, or the SoA state if in < 0.
ep_status sorted_step(ep_ctx *c, const double4 *sub, const double2 *endrot, int K, int in,
                      int out)
{
    if (c->n == 0) {
        return solve_mesh(c, c->mesh(), false);
    }
    const int64_t n4 = (int64_t)c->n >> 2;
    int64_t g = (n4 + kPushBlock - 1) / kPushBlock;
    if (g > c->sort_grid_cap) g = c->sort_grid_cap;
    if (g < 1) g = 1;
    const int grid = (int)g;
    SortArgs a;
    a.zR = c->zR;
    a.zV = c->zV;
    a.ids = c->ids;
    a.rec_in = in >= 0 ? c->rec[in] : nullptr;
    a.n = (int64_t)c->n;
    a.sub = sub;
    a.endrot = endrot;
    a.K = K;
    a.inv_hr = 1.0 / c->hr;
    a.etab = c->etab;
    a.fscal = c->fscal;
    a.nr = (int)c->cfg.n_cells;
    a.counts = c->counts;
    a.total = c->total;
    a.starts = c->starts;
    a.rec_out = c->rec[out];
    a.hist = c->hist;
    a.sums = c->sums;
    HIPCHK(c, timed_launch(c, "sort_count", [&] { return launch_sort_count(c->stream, a, grid); }));
    HIPCHK(c, timed_launch(c, "sort_offsets", [&] { return launch_sort_offsets(c->stream, a, grid); }));
    HIPCHK(c, timed_launch(c, "sort_scatter", [&] { return launch_sort_scatter(c->stream, a, grid); }));
    HIPCHK(c, timed_launch(c, "sort_combine", [&] { return launch_sort_combine(c->stream, a, grid); }));
    return solve_mesh(c, c->mesh(), false);
}

// The records of the last sorted step back to the SoA state (cell order,
// ids with it).
ep_status sorted_unpack(ep_ctx *c, int cur)
{
    c->zR = c->own_zR;
    c->zV = c->own_zV;
    HIPCHK(c, timed_launch(c, "sort_unpack", [&] {
               return launch_sort_unpack(c->stream, c->rec[cur], (int64_t)c->n, c->zR, c->zV,
                                         c->ids);
           }));
    return EP_OK;
}

}  // namespace etd

extern "C" {

const char *ep_last_error(const ep_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

ep_status ep_create(const ep_config *cfg, ep_ctx **out)
{
    if (!out || !cfg) {
        g_create_error = "ep_create: null argument";
        return EP_EINVAL;
    }
    *out = nullptr;
    // The trapezoid scan of the fixed-point charges sums up to 2 N 2^32 in
    // u64, and the learned fallback queue holds 32-bit particle indices: both
    // are exact for N < 2^31.
    if (cfg->n_particles == 0 || cfg->n_particles > kMaxParticles || cfg->substeps == 0 ||
        cfg->n_cells < 2 || (cfg->n_cells & 1) || cfg->n_cells > kMaxCells ||
        !(cfg->r_max > 0.0) || !isfinite(cfg->r_max) ||
        (cfg->deposit != EP_DEPOSIT_ATOMIC && cfg->deposit != EP_DEPOSIT_SORTED)) {
        g_create_error = "ep_create: invalid configuration (need 1 <= n_particles < 2^31, "
                         "substeps >= 1, even 2 <= n_cells <= 8192, r_max > 0, valid deposit)";
        return EP_EINVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) {
        g_create_error = "ep_create: no such HIP device";
        return EP_EINVAL;
    }
    ep_ctx *c = new ep_ctx();
    c->cfg = *cfg;
    c->device = cfg->device;
    c->hr = 2.0 * cfg->r_max / (double)cfg->n_cells;
    DeviceGuard guard(c->device);
    ep_status st = EP_OK;
    auto bail = [&](ep_status s) {
        g_create_error = c->err;
        free_all(c);
        delete c;
        return s;
    };
#define CREATE_CHK(expr)                                  \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) {                           \
            c->hipfail(#expr, e_);                        \
            return bail(e_ == hipErrorOutOfMemory ? EP_ENOMEM : EP_EHIP); \
        }                                                 \
    } while (0)
    if (cfg->hip_stream) {
        c->stream = reinterpret_cast<hipStream_t>(cfg->hip_stream);
    } else {
        CREATE_CHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    hipDeviceProp_t prop;
    CREATE_CHK(hipGetDeviceProperties(&prop, c->device));
    c->n_cu = prop.multiProcessorCount;
    const size_t lds = push_lds_bytes_for((int)cfg->n_cells);
    const size_t lds_cu = prop.maxSharedMemoryPerMultiProcessor ? prop.maxSharedMemoryPerMultiProcessor
                                                                 : 160 * 1024;
    if (lds > prop.sharedMemPerBlock && lds > lds_cu) {
        c->fail(EP_EINVAL, "ep_create: mesh of %u cells needs %zu B of LDS", cfg->n_cells, lds);
        return bail(EP_EINVAL);
    }
    // the sort passes' LDS (up to 20 N_r bytes) fits twice per CU up to
    // N_r = 4096, like the fused push's
    const size_t lds_sort = sort_lds_bytes_for((int)cfg->n_cells);
    int per_cu = (int)(lds_cu / (lds > lds_sort ? lds : lds_sort));
    if (per_cu > 2) per_cu = 2;
    if (per_cu < 1) per_cu = 1;
    // The sort passes keep one counter row per workgroup: the resident
    // workgroups only.  The fused push takes many more workgroups than fit at
    // once, so that the LDS set-up and histogram flush of some overlap the
    // streaming of others (16 per CU measured best at 1e8 particles).
    c->sort_grid_cap = c->n_cu * per_cu;
    c->push_grid_cap = c->n_cu * 16;
    CREATE_CHK(setup_mesh_lds((int)cfg->n_cells));
    CREATE_CHK(setup_learned_lds((int)cfg->n_cells));
    CREATE_CHK(setup_fine_lds((int)cfg->n_cells));

    const size_t np = (size_t)cfg->n_particles;
    const size_t np_pad = (np + 3) & ~size_t(3);
    CREATE_CHK(dalloc(&c->own_zR, np_pad));
    CREATE_CHK(dalloc(&c->own_zV, np_pad));
    c->zR = c->own_zR;
    c->zV = c->own_zV;
    const size_t nn = (size_t)cfg->n_cells + 1;
    if (cfg->deposit == EP_DEPOSIT_SORTED) {
        CREATE_CHK(dalloc(&c->rec[0], 3 * np_pad));
        CREATE_CHK(dalloc(&c->rec[1], 3 * np_pad));
        CREATE_CHK(dalloc(&c->ids, np_pad));
        CREATE_CHK(dalloc(&c->inv, np_pad));
        CREATE_CHK(dalloc(&c->counts, (size_t)c->sort_grid_cap * nn));
        CREATE_CHK(dalloc(&c->sums, (size_t)c->sort_grid_cap * nn));
        CREATE_CHK(dalloc(&c->total, nn));
        CREATE_CHK(dalloc(&c->starts, nn));
        CREATE_CHK(setup_sort_lds((int)cfg->n_cells));
    }
    CREATE_CHK(dalloc(&c->hist, nn));
    CREATE_CHK(dalloc(&c->etab, nn));
    CREATE_CHK(dalloc(&c->rho64, nn));
    CREATE_CHK(dalloc(&c->E64, nn));
    CREATE_CHK(dalloc(&c->Psi64, nn));
    CREATE_CHK(dalloc(&c->fscal, (size_t)kFieldScalars));
    CREATE_CHK(hipMemsetAsync(c->hist, 0, nn * sizeof(unsigned long long), c->stream));
    CREATE_CHK(hipMemsetAsync(c->fscal, 0, kFieldScalars * sizeof(double), c->stream));
    c->mom_grid_cap = moments_grid((int64_t)np);
    CREATE_CHK(dalloc(&c->mpartial, (size_t)c->mom_grid_cap * kMomentQuantities));
    CREATE_CHK(dalloc(&c->mcount, (size_t)c->mom_grid_cap * kMomentCounts));
    CREATE_CHK(dalloc(&c->mout, (size_t)kMomentQuantities));
    CREATE_CHK(dalloc(&c->mout_count, (size_t)kMomentCounts));
    CREATE_CHK(hipStreamSynchronize(c->stream));
#undef CREATE_CHK
    (void)st;
    *out = c;
    return EP_OK;
}

ep_status ep_destroy(ep_ctx *ctx)
{
    if (!ctx) return EP_OK;
    DeviceGuard guard(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    delete ctx;
    return EP_OK;
}

ep_status ep_set_particles(ep_ctx *c, const double *R, const double *V, uint64_t n, double w)
{
    if (!c) return EP_EINVAL;
    if ((n > 0 && (!R || !V)) || n > c->cfg.n_particles || !(w > 0.0) || !isfinite(w))
        return c->fail(EP_EINVAL, "ep_set_particles: need 0 <= n <= capacity (%llu), w > 0",
                       (unsigned long long)c->cfg.n_particles);
    DeviceGuard guard(c->device);
    if (!c->stageR) {
        HIPCHK(c, dalloc(&c->stageR, kStageParticles));
        HIPCHK(c, dalloc(&c->stageV, kStageParticles));
    }
    c->zR = c->own_zR;
    c->zV = c->own_zV;
    const double cs = cos(c->phase), sn = sin(c->phase);
    for (uint64_t off = 0; off < n; off += kStageParticles) {
        const uint64_t m = n - off < kStageParticles ? n - off : kStageParticles;
        HIPCHK(c, hipMemcpyAsync(c->stageR, R + off, m * sizeof(double), hipMemcpyHostToDevice,
                                 c->stream));
        HIPCHK(c, hipMemcpyAsync(c->stageV, V + off, m * sizeof(double), hipMemcpyHostToDevice,
                                 c->stream));
        HIPCHK(c, launch_twist_in(c->stream, c->stageR, c->stageV, c->zR + off, c->zV + off,
                                  (int64_t)m, cs, sn));
        if (c->ids) HIPCHK(c, launch_iota(c->stream, c->ids, (int64_t)off, (int64_t)m));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    c->n = n;
    c->w = w;
    c->field_valid = false;
    c->periods_valid = false;
    return EP_OK;
}

ep_status ep_bind_particles(ep_ctx *c, float *zR_dev, float *zV_dev, uint64_t n, double w)
{
    if (!c) return EP_EINVAL;
    if (c->cfg.deposit == EP_DEPOSIT_SORTED)
        return c->fail(EP_ESTATE, "ep_bind_particles: the sorted deposit reorders particles in "
                                  "library-owned buffers");
    if (!zR_dev || !zV_dev || n > c->cfg.n_particles || !(w > 0.0) ||
        (reinterpret_cast<uintptr_t>(zR_dev) & 15) || (reinterpret_cast<uintptr_t>(zV_dev) & 15))
        return c->fail(EP_EINVAL, "ep_bind_particles: need 16-byte aligned device arrays, "
                                  "n <= capacity, w > 0");
    c->zR = zR_dev;
    c->zV = zV_dev;
    c->n = n;
    c->w = w;
    c->field_valid = false;
    c->periods_valid = false;
    return EP_OK;
}

ep_status ep_step(ep_ctx *c, double dt, double eps, int32_t field, uint64_t n_steps)
{
    if (!c) return EP_EINVAL;
    if (!(dt > 0.0) || !(eps > 0.0) || !isfinite(dt) || !isfinite(eps) ||
        (field != EP_FIELD_ZERO && field != EP_FIELD_DUFFING && field != EP_FIELD_POISSON))
        return c->fail(EP_EINVAL, "ep_step: need dt > 0, eps > 0 and a valid field model");
    if (c->w <= 0.0) return c->fail(EP_ESTATE, "ep_step: no particles loaded");
    if (n_steps == 0) return EP_OK;
    DeviceGuard guard(c->device);
    const int K = (int)c->cfg.substeps;
    const double dphi = fmod(dt / eps, kTwoPi);
    const double theta = dt / ((double)K * eps);
    const double h = dt / (double)K;

    if (field == EP_FIELD_ZERO) {
        // E = 0: the rotating-frame state is unchanged; only the phase advances.
        c->phase = fmod(c->phase + (double)n_steps * dphi, kTwoPi);
        c->t += (double)n_steps * dt;
        c->n_steps += n_steps;
        c->field_valid = false;
        return EP_OK;
    }
    if (c->push_mode == EP_PUSH_LEARNED) return learned_steps(c, dt, eps, field, n_steps);
    if (c->push_mode >= EP_PUSH_RK4) return fine_steps(c, dt, eps, field, n_steps);
    if (field == EP_FIELD_POISSON && !c->field_valid) {
        ep_status s = refresh_field(c);
        if (s != EP_OK) return s;
    }
    size_t chunk = kTableEntries / (size_t)K;
    if (chunk < 1) chunk = 1;
    {
        ep_status s = ensure_tables(c, chunk * (size_t)K < (size_t)K ? (size_t)K : chunk * (size_t)K,
                                    chunk);
        if (s != EP_OK) return s;
    }
    // sorted deposit: the record buffer that holds the state, -1 while it is
    // the SoA state
    int rec_cur = -1;
    uint64_t done = 0;
    while (done < n_steps) {
        const uint64_t rem = n_steps - done;
        const int S = (int)(rem < chunk ? rem : chunk);
        HIPCHK(c, launch_phase_table(c->stream, c->tab, c->phase, dphi, theta, h, K, S));
        if (field == EP_FIELD_DUFFING) {
            HIPCHK(c, timed_launch(c, "push_duffing", [&] {
                       return launch_push_duffing(c->stream, c->zR, c->zV, (int64_t)c->n,
                                                  c->tab.sub, K, S);
                   }));
        } else {
            const MeshArgs ma = c->mesh();
            for (int j = 0; j < S; ++j) {
                if (c->cfg.deposit == EP_DEPOSIT_SORTED) {
                    const int out = rec_cur == 0 ? 1 : 0;
                    ep_status st = sorted_step(c, c->tab.sub + (size_t)j * K, c->tab.endrot + j,
                                               K, rec_cur, out);
                    if (st != EP_OK) {
                        // leave the last completed step's state behind
                        if (rec_cur >= 0) (void)sorted_unpack(c, rec_cur);
                        return st;
                    }
                    if (c->n > 0) rec_cur = out;
                    continue;
                }
                HIPCHK(c, timed_launch(c, "push_poisson", [&] {
                           return launch_push_poisson(c->stream, true, c->zR, c->zV,
                                                      (int64_t)c->n, c->tab.sub + (size_t)j * K,
                                                      c->tab.endrot + j, make_double2(1.0, 0.0),
                                                      K, ma, c->push_grid_cap);
                       }));
                if (ep_status s = solve_mesh(c, ma, false); s != EP_OK) return s;
            }
        }
        c->phase = fmod(c->phase + (double)S * dphi, kTwoPi);
        c->t += (double)S * dt;
        c->n_steps += (uint64_t)S;
        done += (uint64_t)S;
    }
    if (rec_cur >= 0) {
        ep_status s = sorted_unpack(c, rec_cur);
        if (s != EP_OK) return s;
    }
    c->field_valid = (field == EP_FIELD_POISSON);
    return EP_OK;
}

ep_status ep_sync(ep_ctx *c)
{
    if (!c) return EP_EINVAL;
    DeviceGuard guard(c->device);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return EP_OK;
}

ep_status ep_moments_get(ep_ctx *c, double eps, int32_t field, ep_moments *out)
{
    if (!c || !out) return c ? c->fail(EP_EINVAL, "ep_moments_get: null output") : EP_EINVAL;
    if (!(eps > 0.0) ||
        (field != EP_FIELD_ZERO && field != EP_FIELD_DUFFING && field != EP_FIELD_POISSON))
        return c->fail(EP_EINVAL, "ep_moments_get: need eps > 0 and a valid field model");
    if (c->w <= 0.0) return c->fail(EP_ESTATE, "ep_moments_get: no particles loaded");
    DeviceGuard guard(c->device);
    if (field == EP_FIELD_POISSON) {
        ep_status s = c->field_valid ? ensure_potential(c) : refresh_field(c);
        if (s != EP_OK) return s;
    }
    const int grid = moments_grid((int64_t)c->n);
    HIPCHK(c, launch_moments(c->stream, c->zR, c->zV, (int64_t)c->n, cos(c->phase),
                             sin(c->phase), c->cfg.r_max, c->mpartial, c->mcount, grid, c->mout,
                             c->mout_count));
    double q[kMomentQuantities];
    unsigned long long cnt[kMomentCounts];
    double fs[kFieldScalars];
    HIPCHK(c, hipMemcpyAsync(q, c->mout, sizeof q, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(cnt, c->mout_count, sizeof cnt, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(fs, c->fscal, sizeof fs, hipMemcpyDeviceToHost, c->stream));
    unsigned long long fallbacks = 0;
    if (c->mlp.d_total)
        HIPCHK(c, hipMemcpyAsync(&fallbacks, c->mlp.d_total, sizeof fallbacks,
                                 hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const double charge = c->w * (double)c->n;
    out->t = c->t;
    out->phase = c->phase;
    out->charge = charge;
    out->rms_radius = c->n ? sqrt(c->w * q[0] / charge) : 0.0;
    out->kinetic = c->w * q[1] / (2.0 * eps);
    out->potential = field == EP_FIELD_DUFFING ? c->w * q[2] / 4.0
                     : field == EP_FIELD_POISSON ? fs[kFieldEnergy]
                                                 : 0.0;
    out->energy = out->kinetic + out->potential;
    out->n_steps = c->n_steps;
    out->n_offmesh = field == EP_FIELD_POISSON ? cnt[0] : 0;
    out->n_nan = cnt[1];
    out->n_fallback = fallbacks;
    return EP_OK;
}

ep_status ep_get_particles(ep_ctx *c, double *R, double *V, uint64_t offset, uint64_t count)
{
    if (!c) return EP_EINVAL;
    if (offset > c->n || count > c->n - offset || (count > 0 && (!R || !V)))
        return c->fail(EP_EINVAL, "ep_get_particles: range [%llu, +%llu) outside the %llu loaded",
                       (unsigned long long)offset, (unsigned long long)count,
                       (unsigned long long)c->n);
    DeviceGuard guard(c->device);
    if (!c->stageR) {
        HIPCHK(c, dalloc(&c->stageR, kStageParticles));
        HIPCHK(c, dalloc(&c->stageV, kStageParticles));
    }
    const double cs = cos(c->phase), sn = sin(c->phase);
    const bool reordered = c->ids != nullptr;
    if (reordered) HIPCHK(c, launch_inverse(c->stream, c->ids, (int64_t)c->n, c->inv));
    for (uint64_t done = 0; done < count; done += kStageParticles) {
        const uint64_t m = count - done < kStageParticles ? count - done : kStageParticles;
        if (reordered)
            HIPCHK(c, launch_gather_out(c->stream, c->zR, c->zV, c->inv, (int64_t)(offset + done),
                                        (int64_t)m, cs, sn, c->stageR, c->stageV));
        else
            HIPCHK(c, launch_twist_out(c->stream, c->zR + offset + done, c->zV + offset + done,
                                       c->stageR, c->stageV, (int64_t)m, cs, sn));
        HIPCHK(c, hipMemcpyAsync(R + done, c->stageR, m * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipMemcpyAsync(V + done, c->stageV, m * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return EP_OK;
}

ep_status ep_get_field(ep_ctx *c, double *rho, double *E, double *Psi, double *Qb,
                       uint32_t n_nodes)
{
    if (!c) return EP_EINVAL;
    if (n_nodes != c->cfg.n_cells + 1)
        return c->fail(EP_EINVAL, "ep_get_field: n_nodes must be n_cells + 1 = %u",
                       c->cfg.n_cells + 1);
    if (c->w <= 0.0) return c->fail(EP_ESTATE, "ep_get_field: no particles loaded");
    DeviceGuard guard(c->device);
    {
        ep_status s = c->field_valid ? ensure_potential(c) : refresh_field(c);
        if (s != EP_OK) return s;
    }
    const size_t bytes = (size_t)n_nodes * sizeof(double);
    if (rho) HIPCHK(c, hipMemcpyAsync(rho, c->rho64, bytes, hipMemcpyDeviceToHost, c->stream));
    if (E) HIPCHK(c, hipMemcpyAsync(E, c->E64, bytes, hipMemcpyDeviceToHost, c->stream));
    if (Psi) HIPCHK(c, hipMemcpyAsync(Psi, c->Psi64, bytes, hipMemcpyDeviceToHost, c->stream));
    double fs[kFieldScalars];
    HIPCHK(c, hipMemcpyAsync(fs, c->fscal, sizeof fs, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (Qb) *Qb = fs[kQb];
    return EP_OK;
}

ep_status ep_set_push_mode(ep_ctx *c, int32_t push, double drift_tol, uint32_t fallback_substeps)
{
    if (!c) return EP_EINVAL;
    if (push < EP_PUSH_PLAIN || push > EP_PUSH_MODIFIED_ETD)
        return c->fail(EP_EINVAL, "ep_set_push_mode: unknown push mode");
    if (push >= EP_PUSH_RK4 && c->cfg.deposit == EP_DEPOSIT_SORTED)
        return c->fail(EP_EINVAL, "ep_set_push_mode: the fine solvers do not support the sorted "
                                  "deposit");
    if (push == EP_PUSH_LEARNED) {
        if (c->mlp.n_in == 0)
            return c->fail(EP_ENOTRAINED, "ep_set_push_mode: no corrector network loaded");
        if (!(drift_tol >= 0.0) || fallback_substeps == 0)
            return c->fail(EP_EINVAL, "ep_set_push_mode: need drift_tol >= 0 and "
                                      "fallback_substeps >= 1");
        c->drift_tol = drift_tol;
        c->fallback_K = fallback_substeps;
    }
    c->push_mode = push;
    return EP_OK;
}

ep_status ep_copy_bandwidth(int32_t device, uint64_t bytes, int32_t reps, double *gb_per_s)
{
    if (!gb_per_s || bytes == 0 || reps < 1) return EP_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return EP_EINVAL;
    DeviceGuard guard(device);
    void *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ep_status st = EP_EHIP;
    float ms = 0.f;
    if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
        st = EP_ENOMEM;
        goto done;
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) goto done;
    for (int i = 0; i < 3; ++i)
        if (hipMemcpyAsync(b, a, bytes, hipMemcpyDeviceToDevice, nullptr) != hipSuccess) goto done;
    if (hipEventRecord(e0, nullptr) != hipSuccess) goto done;
    for (int i = 0; i < reps; ++i)
        if (hipMemcpyAsync(b, a, bytes, hipMemcpyDeviceToDevice, nullptr) != hipSuccess) goto done;
    if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0.f))
        goto done;
    *gb_per_s = 2.0 * (double)bytes * reps / ((double)ms / 1e3) / 1e9;
    st = EP_OK;
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    return st;
}

ep_status ep_timing_enable(ep_ctx *c, int32_t on)
{
    if (!c) return EP_EINVAL;
    if (on < 0) return c->fail(EP_EINVAL, "ep_timing_enable: on must be >= 0, not %d", (int)on);
    DeviceGuard guard(c->device);
    HIPCHK(c, collect_timing(c));
    c->timed.clear();
    c->launch_seq.clear();
    c->timing = on != 0;
    c->timing_stride = on > 1 ? (uint32_t)on : 1u;
    return EP_OK;
}

ep_status ep_timing_get(ep_ctx *c, const char *kernel, double *total_ms, uint64_t *count)
{
    if (!c) return EP_EINVAL;
    if (!kernel || !total_ms || !count) return c->fail(EP_EINVAL, "ep_timing_get: null argument");
    DeviceGuard guard(c->device);
    HIPCHK(c, collect_timing(c));
    auto it = c->timed.find(kernel);
    *total_ms = it == c->timed.end() ? 0.0 : it->second.first;
    *count = it == c->timed.end() ? 0 : it->second.second;
    return EP_OK;
}

}  // extern "C"
