// Checkpoint and resume of a context (ep_save / ep_load).

#include "context.h"

using namespace etd;

namespace {

constexpr char kMagic[8] = {'E', 'T', 'D', 'P', 'I', 'C', '0', '1'};
constexpr uint32_t kVersion = 4;   // 4: normalisation of 9 values (base push)

struct Header {
    char magic[8];
    uint32_t version;
    uint32_t n_cells;
    uint64_t n;
    uint32_t substeps;
    int32_t deposit;
    double r_max;
    double w;
    double t;
    double phase;
    uint64_t n_steps;
    int32_t push_mode;
    uint32_t fallback_K;
    double drift_tol;
    uint32_t mlp_n_in;
    uint32_t mlp_n_params;
    int32_t mlp_precision;
    uint32_t mlp_project;       // 1: energy projection of the learned push
    double h_fine;
    uint64_t max_fine;
    int32_t periods_once;
    int32_t periods_saved;      // 1: the periods T_i and N_i follow the particles
    int32_t periods_duffing;    // 1: reusable Duffing periods
    uint32_t reserved2;
    double periods_eps;
    double periods_h;
    uint64_t periods_unresolved;
};

struct File {
    FILE *f = nullptr;
    ~File()
    {
        if (f) fclose(f);
    }
};

}  // namespace

extern "C" {

ep_status ep_save(ep_ctx *c, const char *path)
{
    if (!c) return EP_EINVAL;
    if (!path) return c->fail(EP_EINVAL, "ep_save: null path");
    DeviceGuard guard(c->device);
    Header h{};
    memcpy(h.magic, kMagic, 8);
    h.version = kVersion;
    h.n_cells = c->cfg.n_cells;
    h.n = c->n;
    h.substeps = c->cfg.substeps;
    h.deposit = c->cfg.deposit;
    h.r_max = c->cfg.r_max;
    h.w = c->w;
    h.t = c->t;
    h.phase = c->phase;
    h.n_steps = c->n_steps;
    h.push_mode = c->push_mode;
    h.fallback_K = c->fallback_K;
    h.drift_tol = c->drift_tol;
    h.mlp_n_in = (uint32_t)c->mlp.n_in;
    h.mlp_n_params = (uint32_t)c->mlp.params.size();
    h.mlp_precision = c->mlp.precision;
    h.mlp_project = c->mlp.project ? 1u : 0u;
    h.h_fine = c->h_fine;
    h.max_fine = c->max_fine;
    h.periods_once = c->periods_once ? 1 : 0;
    // periods of the last period-finding step, if they belong to these particles
    std::vector<double> T;
    std::vector<int64_t> N;
    if (c->periods_valid && !c->ids && c->n && c->fine.T) {
        T.resize(c->n);
        N.resize(c->n);
        unsigned long long un = 0;
        HIPCHK(c, hipMemcpyAsync(T.data(), c->fine.T, c->n * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(N.data(), c->fine.N, c->n * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(&un, c->fine.unresolved, sizeof un, hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        h.periods_saved = 1;
        h.periods_duffing = c->periods_duffing && c->periods_step == c->n_steps ? 1 : 0;
        h.periods_eps = c->periods_eps;
        h.periods_h = c->periods_h;
        h.periods_unresolved = un;
    }
    // particles in loaded order
    std::vector<float> zr(c->n), zv(c->n);
    if (c->n) {
        if (c->ids) {
            HIPCHK(c, launch_inverse(c->stream, c->ids, (int64_t)c->n, c->inv));
            float *tmpR = nullptr, *tmpV = nullptr;
            HIPCHK(c, dalloc(&tmpR, (size_t)c->n));
            HIPCHK(c, dalloc(&tmpV, (size_t)c->n));
            hipError_t e = launch_gather_f32(c->stream, c->zR, c->zV, c->inv, (int64_t)c->n, tmpR,
                                             tmpV);
            if (e == hipSuccess)
                e = hipMemcpyAsync(zr.data(), tmpR, c->n * 4, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(zv.data(), tmpV, c->n * 4, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            (void)hipFree(tmpR);
            (void)hipFree(tmpV);
            if (e != hipSuccess) return c->hipfail("ep_save: gather particles", e);
        } else {
            HIPCHK(c, hipMemcpyAsync(zr.data(), c->zR, c->n * 4, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipMemcpyAsync(zv.data(), c->zV, c->n * 4, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
    }
    File out;
    out.f = fopen(path, "wb");
    if (!out.f) return c->fail(EP_EIO, "ep_save: cannot open %s", path);
    bool ok = fwrite(&h, sizeof h, 1, out.f) == 1;
    if (c->n) {
        ok = ok && fwrite(zr.data(), 4, c->n, out.f) == c->n;
        ok = ok && fwrite(zv.data(), 4, c->n, out.f) == c->n;
    }
    if (h.mlp_n_in) {
        ok = ok && fwrite(c->mlp.params.data(), 4, h.mlp_n_params, out.f) == h.mlp_n_params;
        ok = ok && fwrite(c->mlp.norm, 8, kNormLen, out.f) == (size_t)kNormLen;
    }
    if (h.periods_saved) {
        ok = ok && fwrite(T.data(), 8, c->n, out.f) == c->n;
        ok = ok && fwrite(N.data(), 8, c->n, out.f) == c->n;
    }
    ok = ok && fflush(out.f) == 0;
    if (!ok) return c->fail(EP_EIO, "ep_save: write to %s failed", path);
    return EP_OK;
}

ep_status ep_load(ep_ctx *c, const char *path, uint64_t *n_particles)
{
    if (!c) return EP_EINVAL;
    if (!path) return c->fail(EP_EINVAL, "ep_load: null path");
    File in;
    in.f = fopen(path, "rb");
    if (!in.f) return c->fail(EP_EIO, "ep_load: cannot open %s", path);
    Header h{};
    if (fread(&h, sizeof h, 1, in.f) != 1 || memcmp(h.magic, kMagic, 8) != 0 ||
        h.version != kVersion)
        return c->fail(EP_EIO, "ep_load: %s is not a checkpoint of format %u", path, kVersion);
    if (h.n > c->cfg.n_particles || h.n_cells != c->cfg.n_cells || h.r_max != c->cfg.r_max ||
        h.substeps != c->cfg.substeps || !(h.w > 0.0) ||
        (h.mlp_n_in && h.mlp_n_params != (uint32_t)mlp_n_params((int)h.mlp_n_in)))
        return c->fail(EP_EINVAL, "ep_load: checkpoint does not fit this context (particles, "
                                  "mesh or substeps differ)");
    // the learned push's settings obey the bounds of ep_set_push_mode
    if (!(h.drift_tol >= 0.0) || (h.push_mode == EP_PUSH_LEARNED && h.fallback_K == 0))
        return c->fail(EP_EINVAL, "ep_load: checkpoint has an invalid drift bound or fallback "
                                  "substep count");
    std::vector<float> zr(h.n), zv(h.n), params(h.mlp_n_params);
    std::vector<double> T(h.periods_saved ? h.n : 0);
    std::vector<int64_t> N(h.periods_saved ? h.n : 0);
    double norm[kNormLen] = {0};
    bool ok = true;
    if (h.n) {
        ok = fread(zr.data(), 4, h.n, in.f) == h.n && fread(zv.data(), 4, h.n, in.f) == h.n;
    }
    if (ok && h.mlp_n_in)
        ok = fread(params.data(), 4, h.mlp_n_params, in.f) == h.mlp_n_params &&
             fread(norm, 8, kNormLen, in.f) == (size_t)kNormLen;
    if (ok && h.periods_saved)
        ok = fread(T.data(), 8, h.n, in.f) == h.n && fread(N.data(), 8, h.n, in.f) == h.n;
    if (!ok) return c->fail(EP_EIO, "ep_load: %s is truncated", path);
    DeviceGuard guard(c->device);
    if (h.mlp_n_in) {
        ep_status s = ep_mlp_set_weights(c, params.data(), h.mlp_n_params, norm);
        if (s != EP_OK) return s;
    }
    c->zR = c->own_zR;
    c->zV = c->own_zV;
    if (h.n) {
        HIPCHK(c, copy_sync(c, c->zR, zr.data(), h.n * 4, hipMemcpyHostToDevice));
        HIPCHK(c, copy_sync(c, c->zV, zv.data(), h.n * 4, hipMemcpyHostToDevice));
        if (c->ids) HIPCHK(c, launch_iota(c->stream, c->ids, 0, (int64_t)h.n));
    }
    c->n = h.n;
    c->w = h.w;
    c->t = h.t;
    c->phase = h.phase;
    c->n_steps = h.n_steps;
    // the push mode as saved, where this context supports it (else plain)
    int32_t mode = h.push_mode;
    if (mode < EP_PUSH_PLAIN || mode > EP_PUSH_MODIFIED_ETD) mode = EP_PUSH_PLAIN;
    if (mode == EP_PUSH_LEARNED && !c->mlp.n_in) mode = EP_PUSH_PLAIN;
    if (mode >= EP_PUSH_RK4 && c->cfg.deposit == EP_DEPOSIT_SORTED) mode = EP_PUSH_PLAIN;
    c->push_mode = mode;
    if (h.mlp_precision == EP_MLP_BF16 || h.mlp_precision == EP_MLP_FP16)
        (void)ep_mlp_set_precision(c, h.mlp_precision);
    (void)ep_mlp_set_projection(c, h.mlp_project == 1 ? 1 : 0);
    if (isfinite(h.h_fine) && h.max_fine >= 1) {
        c->h_fine = h.h_fine;
        c->max_fine = h.max_fine;
    }
    c->fallback_K = h.fallback_K;
    c->drift_tol = h.drift_tol;
    c->periods_once = h.periods_once != 0;
    c->field_valid = false;
    c->periods_valid = false;
    c->periods_duffing = false;
    if (h.periods_saved && h.n) {
        ep_status s = restore_periods(c, T.data(), N.data(), h.periods_unresolved);
        if (s != EP_OK) return s;
        c->periods_valid = true;
        c->periods_duffing = h.periods_duffing != 0;
        c->periods_eps = h.periods_eps;
        c->periods_h = h.periods_h;
        c->periods_step = c->n_steps;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (n_particles) *n_particles = h.n;
    return EP_OK;
}

}  // extern "C"
