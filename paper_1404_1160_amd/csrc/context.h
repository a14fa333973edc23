// Context of the etdpic library: device buffers, clock, push mode and the
// learned corrector's state; shared by the host runtime translation units.
#pragma once

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/etdpic.h"
#include "internal.h"

namespace etd {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr uint32_t kMaxCells = 8192;
constexpr uint64_t kMaxParticles = (uint64_t(1) << 31) - 1;
constexpr size_t kTableEntries = size_t(1) << 20;   // substep coefficients per chunk
constexpr size_t kStageParticles = size_t(1) << 23; // FP64 staging for host transfers

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

template <typename T>
hipError_t dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
}

// Normalisation of a trained corrector: {s_in, s_t, s_E, mu_d, sig_d, mu_k,
// sig_k, output map, base substeps}.
constexpr int kNormLen = 9;
constexpr uint32_t kMaxBaseK = 4096;   // substeps of a base push

// Learned corrector state.
struct Learned {
    int n_in = 0;                    // 0: no network loaded
    std::vector<float> params;       // FP32 master copy (host)
    double norm[kNormLen] = {0};
    float *d_params = nullptr, *d_m = nullptr, *d_v = nullptr, *d_grad = nullptr;
    // inference constants for (dt, eps) = cached_dt, cached_eps
    uint4 *d_w1f = nullptr, *d_w2f = nullptr;
    int32_t precision = EP_MLP_BF16;   // MFMA operand type of the inference
    bool project = false;              // energy projection of the passing particles
    float4 *d_b2 = nullptr;
    uint4 *d_w3f = nullptr;
    bool packed = false;
    double cached_dt = -1.0, cached_eps = -1.0;
    MlpInfer infer{};
    // fallback queue
    unsigned *d_qcount = nullptr, *d_queue = nullptr;
    unsigned long long *d_total = nullptr;
    uint64_t queue_cap = 0;
    // training set collected from the context's own particles (features
    // [t_n][6], raw labels [t_n][2])
    float *d_tx = nullptr, *d_ty = nullptr;
    uint64_t t_n = 0, t_cap = 0;
    // base push (norm[8] > 0): its substep coefficients and its result
    StepTables btab{};
    size_t btab_cap = 0;
    float *d_cR = nullptr, *d_cV = nullptr;
    uint64_t base_cap = 0;
};

}  // namespace etd

using etd::Learned;
using etd::MeshArgs;
using etd::StepTables;

struct ep_ctx {
    etd::Learned mlp;
    ep_config cfg{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int n_cu = 0;
    int push_grid_cap = 0;           // workgroups of the fused Poisson push
    int sort_grid_cap = 0;           // workgroups of the sort passes (resident ones)

    // particle state (rotating frame, FP32 SoA)
    float *zR = nullptr, *zV = nullptr;
    float *own_zR = nullptr, *own_zV = nullptr;
    uint64_t n = 0;
    double w = 0.0;

    // mesh
    double hr = 0.0;
    unsigned long long *hist = nullptr;
    float2 *etab = nullptr;
    double *rho64 = nullptr, *E64 = nullptr, *Psi64 = nullptr, *fscal = nullptr;
    bool field_valid = false;
    bool potential_valid = false;   // Psi64 and the field energy belong to the field

    MeshArgs mesh() const
    {
        MeshArgs m;
        m.nr = (int)cfg.n_cells;
        m.w = w;
        m.hr = hr;
        m.hist = hist;
        m.etab = etab;
        m.rho64 = rho64;
        m.E64 = E64;
        m.Psi64 = Psi64;
        m.fscal = fscal;
        return m;
    }

    // sorted deposit: the state as records within a call (two buffers, cell
    // order), ids, count tables
    unsigned *rec[2] = {nullptr, nullptr};   // (R, V, id) records, 12 B per particle
    unsigned *ids = nullptr, *inv = nullptr;
    unsigned *counts = nullptr, *total = nullptr, *starts = nullptr;
    unsigned long long *sums = nullptr;   // segment sums of the scatter pass [grid][nr+1]

    // per-chunk substep tables
    StepTables tab{};
    size_t tab_cap = 0;

    // host transfers
    double *stageR = nullptr, *stageV = nullptr;

    // moments
    int mom_grid_cap = 0;
    double *mpartial = nullptr, *mout = nullptr;
    unsigned long long *mcount = nullptr, *mout_count = nullptr;

    // clock: t and the fast phase t/eps mod 2 pi, FP64
    double t = 0.0, phase = 0.0;
    uint64_t n_steps = 0;

    // fine solvers (reference RK4, improved ETD)
    double h_fine = 0.0;
    uint64_t max_fine = 10000;
    etd::FineArgs fine{};
    uint64_t fine_cap = 0;
    bool periods_valid = false;
    double last_period = 0.0;        // common period P of the last classic/modified ETD step
    // In the given (Duffing) field each particle's period is constant, so the
    // periods found once are reused by later improved ETD steps (section 3)
    // while nothing but period-finding steps has moved the particles.
    bool periods_once = true;
    bool periods_duffing = false;    // fine.T holds Duffing periods of the current particles
    double periods_eps = 0.0, periods_h = 0.0;
    uint64_t periods_step = 0;       // n_steps when they were last found or used

    // push mode
    int push_mode = EP_PUSH_PLAIN;
    double drift_tol = 1e-5;
    uint32_t fallback_K = 0;

    // timing (every timing_stride-th launch of each kernel name)
    bool timing = false;
    uint32_t timing_stride = 1;
    std::map<std::string, uint64_t> launch_seq;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> event_pool;
    std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::map<std::string, std::pair<double, uint64_t>> timed;

    std::string err;

    ep_status fail(ep_status code, const char *fmt, ...)
    {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
    ep_status hipfail(const char *what, hipError_t e)
    {
        return fail(EP_EHIP, "%s: %s", what, hipGetErrorString(e));
    }
};

#define HIPCHK(ctx, expr)                                   \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return (ctx)->hipfail(#expr, e_); \
    } while (0)

namespace etd {

// Timed launch bracket: records events around `launch` when timing is on,
// for every timing_stride-th launch of each kernel name.
template <typename F>
inline hipError_t timed_launch(ep_ctx *c, const char *name, F &&launch)
{
    if (!c->timing) return launch();
    if (c->timing_stride > 1 && c->launch_seq[name]++ % c->timing_stride != 0) return launch();
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (!c->event_pool.empty()) {
        ev = c->event_pool.back();
        c->event_pool.pop_back();
    } else {
        hipError_t e = hipEventCreate(&ev.first);
        if (e != hipSuccess) return e;
        e = hipEventCreate(&ev.second);
        if (e != hipSuccess) return e;
    }
    etd::LaunchEvents &le = etd::next_launch_events();
    le.start = ev.first;
    le.stop = ev.second;
    hipError_t e = launch();
    const bool consumed = le.start == nullptr && le.stop == nullptr;
    le = etd::LaunchEvents();
    if (e != hipSuccess) return e;
    // every timed launcher dispatches through dispatch_k, which takes both
    if (!consumed) return hipErrorNotSupported;
    c->pending.emplace_back(name, ev);
    return hipSuccess;
}

// Copy on the context's stream and wait for it: the copy follows every
// kernel already queued there (the library's own stream does not synchronise
// with the null stream, so a plain hipMemcpy could overwrite buffers that a
// queued step still reads, or read results it has not yet written), and the
// host buffer is free again when this returns.
inline hipError_t copy_sync(ep_ctx *c, void *dst, const void *src, size_t bytes,
                            hipMemcpyKind kind)
{
    hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, c->stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(c->stream);
}

// Message that ep_last_error(NULL) returns: the last failed call that has no
// context (ep_create, ep_step_noalloc).
void set_context_free_error(const char *msg);
hipError_t collect_timing(ep_ctx *c);
ep_status ensure_tables(ep_ctx *c, size_t entries, size_t steps);
ep_status refresh_field(ep_ctx *c);
// Field of the accumulated charge; with potential also Psi and the field
// energy, which only the learned Poisson push, the moments and ep_get_field
// read.
ep_status solve_mesh(ep_ctx *c, const MeshArgs &ma, bool potential);
// Psi and the field energy of the current field, if a solve left them out.
ep_status ensure_potential(ep_ctx *c);
ep_status sorted_step(ep_ctx *c, const double4 *sub, const double2 *endrot, int K, int in,
                      int out);
ep_status sorted_unpack(ep_ctx *c, int cur);
void free_learned(ep_ctx *c);
// Learned push of n_steps steps (Duffing field); defined with the learned API.
ep_status learned_steps(ep_ctx *c, double dt, double eps, int32_t field, uint64_t n_steps);
// Reference RK4 or improved ETD steps (push modes EP_PUSH_RK4 / _IMPROVED_ETD).
ep_status fine_steps(ep_ctx *c, double dt, double eps, int32_t field, uint64_t n_steps);
void free_fine(ep_ctx *c);
// Duffing periods into fine.T and fine.N (checkpoint restore)
ep_status restore_periods(ep_ctx *c, const double *T, const int64_t *N, uint64_t unresolved);

}  // namespace etd
