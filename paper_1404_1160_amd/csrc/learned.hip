// Host side of the learned Duhamel corrector: parameters, label generation,
// training loop (Adam, cosine-decayed step size), inference constants and the
// learned step with energy check and plain fallback.

#include "context.h"

using namespace etd;

namespace {

constexpr double kAdamB1 = 0.9, kAdamB2 = 0.999, kAdamEps = 1e-8;
constexpr double kTimeScale = 100.0;   // s_t: feature scale of dt/eps
constexpr uint32_t kNormSamples = 65536;

// FP32 -> FP16 bits, round to nearest even (subnormals, overflow to inf).
uint16_t host_f16(float f)
{
    uint32_t x;
    memcpy(&x, &f, 4);
    const uint32_t sign = (x >> 16) & 0x8000u, ax = x & 0x7FFFFFFFu;
    if (ax > 0x7F800000u) return (uint16_t)(sign | 0x7E00u);
    if (ax >= 0x477FF000u) return (uint16_t)(sign | 0x7C00u);
    if (ax < 0x38800000u) {
        float v;
        memcpy(&v, &ax, 4);
        return (uint16_t)(sign | (uint32_t)nearbyintf(v * 16777216.0f));
    }
    const uint32_t m = ax + 0xFFFu + ((ax >> 13) & 1u) - (112u << 23);
    return (uint16_t)(sign | (m >> 13));
}

float host_f16_value(uint16_t h)
{
    const uint32_t e = (h >> 10) & 0x1Fu, m = h & 0x3FFu;
    float v;
    if (e == 0) {
        v = (float)m * (1.0f / 16777216.0f);
    } else if (e == 31) {
        v = m ? NAN : INFINITY;
    } else {
        const uint32_t b = ((e + 112u) << 23) | (m << 13);
        memcpy(&v, &b, 4);
    }
    return (h & 0x8000u) ? -v : v;
}

// FP32 -> BF16 bits, round to nearest even.
uint16_t host_bf16(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);   // NaN stays NaN
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

float host_bf16_value(uint16_t b)
{
    const uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// w as hi + lo in FP16 (fp16 != 0, ~22 significant bits together) or BF16
// (~16 bits); lo = round(w - hi)
void split_op(int fp16, float w, uint16_t &hi, uint16_t &lo)
{
    if (fp16) {
        hi = host_f16(w);
        lo = host_f16(w - host_f16_value(hi));
    } else {
        hi = host_bf16(w);
        lo = host_bf16(w - host_bf16_value(hi));
    }
}

struct Offsets {
    int W1, b1, W2, b2, W3, b3, total;
};

Offsets offsets(int n_in)
{
    Offsets o;
    o.W1 = 0;
    o.b1 = kH * n_in;
    o.W2 = o.b1 + kH;
    o.b2 = o.W2 + kH * kH;
    o.W3 = o.b2 + kH;
    o.b3 = o.W3 + kOut * kH;
    o.total = o.b3 + kOut;
    return o;
}

ep_status ensure_mlp_buffers(ep_ctx *c, int n_in)
{
    Learned &L = c->mlp;
    if (L.d_params && L.n_in == n_in) return EP_OK;
    free_learned(c);
    const size_t np = (size_t)mlp_n_params(n_in);
    HIPCHK(c, dalloc(&L.d_params, np));
    HIPCHK(c, dalloc(&L.d_m, np));
    HIPCHK(c, dalloc(&L.d_v, np));
    HIPCHK(c, dalloc(&L.d_grad, np));
    HIPCHK(c, dalloc(&L.d_w2f, (size_t)2 * 8 * 64));
    HIPCHK(c, dalloc(&L.d_w1f, (size_t)2 * 64));
    HIPCHK(c, dalloc(&L.d_b2, (size_t)kH / 4));
    HIPCHK(c, dalloc(&L.d_w3f, (size_t)2 * 4 * 64));
    HIPCHK(c, dalloc(&L.d_qcount, (size_t)1));
    HIPCHK(c, dalloc(&L.d_total, (size_t)1));
    HIPCHK(c, hipMemsetAsync(L.d_total, 0, sizeof(unsigned long long), c->stream));
    L.n_in = n_in;
    return EP_OK;
}

// Hidden unit that MFMA operand slot (k step kk, lane group g, element e)
// stands for: the unit whose result lane (., g) holds in accumulator element
// 8 (kk % 2) + e of tile kk / 2, so that one layer's results are the next
// layer's B operand as they sit in the lanes.
int slot_unit(int kk, int g, int e)
{
    return 32 * (kk >> 1) + 16 * (kk & 1) + 8 * (e >> 2) + 4 * g + (e & 3);
}

// Inference constants for one (dt, eps), as MFMA A-fragments in the chosen
// operand type (lane l: row l % 32, k = 8 (l / 32) + e of the step): layer 1
// as split hi + lo with the constant features folded into the bias, W2 and
// the biases scaled by 1/64 (the activation takes z / 64), W2 and W3 in
// slot_unit order (with BF16 also their lo parts).  With FP16, fails if a
// pre-activation could leave the activation's FP16 range.
ep_status prepare_inference(ep_ctx *c, double dt, double eps)
{
    Learned &L = c->mlp;
    if (L.packed && L.cached_dt == dt && L.cached_eps == eps) return EP_OK;
    const int fp16 = L.precision == EP_MLP_FP16 ? 1 : 0;
    const Offsets o = offsets(L.n_in);
    const float *P = L.params.data();
    constexpr double kPre = 1.0 / 64.0, kUMax = 255.0;   // |z / 64| < 255: u^2 finite
    const double s_in = L.norm[0], s_t = L.norm[1], s_E = L.norm[2];
    const double th = dt / eps;
    const double phi = fmod(th, kTwoPi);

    // layer 1: per unit (w_R, w_V, w_E, b') / 64
    std::vector<uint16_t> w1((size_t)2 * 64 * 8, 0);
    double xmax = 30000.0;   // keeps the features' FP16 parts finite
    for (int u = 0; u < kH; ++u) {
        const float *w = P + o.W1 + u * L.n_in;
        const double b = (double)P[o.b1 + u] + (double)w[2] * cos(phi) + (double)w[3] * sin(phi) +
                         (double)w[4] * th / s_t;
        const double wf[4] = {w[0] / s_in * kPre, w[1] / s_in * kPre,
                              L.n_in == 6 ? w[5] / s_E * kPre : 0.0, b * kPre};
        const double room = kUMax - fabs(wf[3]), slope = fabs(wf[0]) + fabs(wf[1]) + fabs(wf[2]);
        if (fp16) {
            if (!(room > 0.0))
                return c->fail(EP_EINVAL, "network bias too large for the FP16 inference path");
            if (slope > 0.0) xmax = fmin(xmax, room / slope);
        }
        const int t = u >> 5, i = u & 31;
        for (int f = 0; f < 4; ++f) {
            uint16_t hi, lo;
            split_op(fp16, (float)wf[f], hi, lo);
            w1[((size_t)t * 64 + i) * 8 + f] = hi;                 // g = 0: hi x (x_hi, 1)
            if (f < 3) w1[((size_t)t * 64 + i) * 8 + 4 + f] = hi;  //        hi x x_lo
            w1[((size_t)t * 64 + 32 + i) * 8 + f] = lo;            // g = 1: lo x (x_hi, 1)
        }
    }
    if (fp16 && !(xmax >= 1.0))
        return c->fail(EP_EINVAL, "network weights too large for the FP16 inference path");

    // layer 2
    constexpr size_t kW2 = (size_t)8 * 64 * 8, kW3 = (size_t)4 * 64 * 8;   // values per part
    std::vector<uint16_t> w2(2 * kW2, 0);
    for (int mt = 0; mt < 2; ++mt)
        for (int kk = 0; kk < 4; ++kk)
            for (int lane = 0; lane < 64; ++lane)
                for (int e = 0; e < 8; ++e) {
                    const int i = mt * 32 + (lane & 31), k = slot_unit(kk, lane >> 5, e);
                    const size_t at = ((size_t)(mt * 4 + kk) * 64 + lane) * 8 + e;
                    split_op(fp16, (float)(P[o.W2 + i * kH + k] * kPre), w2[at], w2[kW2 + at]);
                }
    std::vector<float> b2(kH);
    for (int j = 0; j < kH; ++j) {
        double bound = fabs((double)P[o.b2 + j]);
        for (int k = 0; k < kH; ++k) bound += fabs((double)P[o.W2 + j * kH + k]);
        if (fp16 && !(bound * kPre < kUMax))
            return c->fail(EP_EINVAL, "network weights too large for the FP16 inference path");
        b2[j] = (float)(P[o.b2 + j] * kPre);
    }
    // layer 3: rows 0 and 1 are the outputs, the rest zero
    std::vector<uint16_t> w3(2 * kW3, 0);
    for (int kk = 0; kk < 4; ++kk)
        for (int lane = 0; lane < 64; ++lane)
            for (int e = 0; e < 8; ++e) {
                const int i = lane & 31;
                const size_t at = ((size_t)kk * 64 + lane) * 8 + e;
                if (i < kOut)
                    split_op(fp16, P[o.W3 + i * kH + slot_unit(kk, lane >> 5, e)], w3[at],
                             w3[kW3 + at]);
            }
    HIPCHK(c, copy_sync(c, L.d_w1f, w1.data(), w1.size() * 2, hipMemcpyHostToDevice));
    HIPCHK(c, copy_sync(c, L.d_w2f, w2.data(), w2.size() * 2, hipMemcpyHostToDevice));
    HIPCHK(c, copy_sync(c, L.d_b2, b2.data(), kH * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(c, copy_sync(c, L.d_w3f, w3.data(), w3.size() * 2, hipMemcpyHostToDevice));
    MlpInfer &I = L.infer;
    I.w1f = L.d_w1f;
    I.w2f = L.d_w2f;
    I.b2 = L.d_b2;
    I.w3f = L.d_w3f;
    I.b3_0 = P[o.b3];
    I.b3_1 = P[o.b3 + 1];
    I.mu_d = (float)L.norm[3];
    I.sig_d = (float)L.norm[4];
    I.mu_k = (float)L.norm[5];
    I.sig_k = (float)L.norm[6];
    I.xmax = (float)xmax;
    I.fp16 = fp16;
    I.scaled = L.norm[7] == 1.0 ? 1 : 0;
    I.project = L.project ? 1 : 0;
    L.packed = true;
    L.cached_dt = dt;
    L.cached_eps = eps;
    return EP_OK;
}

ep_status ensure_queue(ep_ctx *c)
{
    Learned &L = c->mlp;
    if (L.queue_cap >= c->n && L.d_queue) return EP_OK;
    if (L.d_queue) (void)hipFree(L.d_queue);
    L.d_queue = nullptr;
    L.queue_cap = 0;
    HIPCHK(c, dalloc(&L.d_queue, (size_t)c->n));
    L.queue_cap = c->n;
    return EP_OK;
}

template <typename T>
struct DevBuf {
    T *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

struct Events {
    hipEvent_t e[3] = {nullptr, nullptr, nullptr};
    ~Events()
    {
        for (hipEvent_t x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

// Substep table of the base push for `steps` steps of Kb substeps, and the
// base arrays for the loaded particles.
ep_status ensure_base(ep_ctx *c, size_t entries, size_t steps, bool arrays)
{
    Learned &L = c->mlp;
    if (entries > L.btab_cap || steps > L.btab_cap) {
        size_t cap = entries > steps ? entries : steps;
        if (cap < 1024) cap = 1024;
        if (L.btab.sub) (void)hipFree(L.btab.sub);
        if (L.btab.endrot) (void)hipFree(L.btab.endrot);
        L.btab = StepTables{};
        L.btab_cap = 0;
        HIPCHK(c, dalloc(&L.btab.sub, cap));
        HIPCHK(c, dalloc(&L.btab.endrot, cap));
        L.btab_cap = cap;
    }
    if (arrays && L.base_cap < c->n) {
        if (L.d_cR) (void)hipFree(L.d_cR);
        if (L.d_cV) (void)hipFree(L.d_cV);
        L.d_cR = L.d_cV = nullptr;
        L.base_cap = 0;
        HIPCHK(c, dalloc(&L.d_cR, (size_t)c->n));
        HIPCHK(c, dalloc(&L.d_cV, (size_t)c->n));
        L.base_cap = c->n;
    }
    return EP_OK;
}

// Substeps of the loaded network's base push (0: none, or no network).
int base_substeps(const ep_ctx *c) { return c->mlp.n_in ? (int)c->mlp.norm[8] : 0; }

ep_status upload_fp32(ep_ctx *c, const double *src, uint64_t n, float *dst)
{
    std::vector<float> tmp(n);
    for (uint64_t i = 0; i < n; ++i) tmp[i] = (float)src[i];
    HIPCHK(c, copy_sync(c, dst, tmp.data(), n * sizeof(float), hipMemcpyHostToDevice));
    return EP_OK;
}

// Features and raw labels of n samples into device arrays X[n][5], Y[n][2],
// around the plain push with Kb substeps when Kb > 0.
ep_status make_labels(ep_ctx *c, double dt, double eps, uint32_t K, int Kb, double s_in,
                      int scaled, const double *R, const double *V, uint64_t n, float *dX,
                      float *dY)
{
    DevBuf<float> dR, dV;
    HIPCHK(c, dalloc(&dR.p, (size_t)n));
    HIPCHK(c, dalloc(&dV.p, (size_t)n));
    ep_status s = upload_fp32(c, R, n, dR.p);
    if (s != EP_OK) return s;
    if ((s = upload_fp32(c, V, n, dV.p)) != EP_OK) return s;
    if ((s = ensure_tables(c, K, 1)) != EP_OK) return s;
    if (Kb > 0 && (s = ensure_base(c, (size_t)Kb, 1, false)) != EP_OK) return s;
    const double th = dt / eps;
    HIPCHK(c, launch_phase_table(c->stream, c->tab, 0.0, fmod(th, kTwoPi), th / K, dt / K, (int)K, 1));
    if (Kb > 0)
        HIPCHK(c, launch_phase_table(c->stream, c->mlp.btab, 0.0, fmod(th, kTwoPi), th / Kb,
                                     dt / Kb, Kb, 1));
    const double phi = fmod(th, kTwoPi);
    HIPCHK(c, launch_gen_labels_duffing(c->stream, dR.p, dV.p, (int64_t)n, c->tab.sub, (int)K,
                                        c->mlp.btab.sub, Kb, (float)(1.0 / s_in), (float)cos(phi),
                                        (float)sin(phi), (float)(th / kTimeScale), scaled, dX,
                                        dY));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return EP_OK;
}

}  // namespace

namespace etd {

void free_learned(ep_ctx *c)
{
    Learned &L = c->mlp;
    for (void *p : {(void *)L.d_params, (void *)L.d_m, (void *)L.d_v, (void *)L.d_grad,
                    (void *)L.d_w2f, (void *)L.d_w1f, (void *)L.d_b2,
                    (void *)L.d_w3f, (void *)L.d_qcount, (void *)L.d_queue, (void *)L.d_total,
                    (void *)L.d_tx, (void *)L.d_ty, (void *)L.btab.sub, (void *)L.btab.endrot,
                    (void *)L.d_cR, (void *)L.d_cV})
        if (p) (void)hipFree(p);
    // settings of the context, not of the network
    const int32_t precision = L.precision;
    const bool project = L.project;
    L = Learned();
    L.precision = precision;
    L.project = project;
}

ep_status learned_steps(ep_ctx *c, double dt, double eps, int32_t field, uint64_t n_steps)
{
    Learned &L = c->mlp;
    const bool vp = field == EP_FIELD_POISSON;
    if (L.n_in != (vp ? 6 : 5))
        return c->fail(EP_ENOTRAINED, vp ? "ep_step: the learned push in the Poisson field needs "
                                           "a 6-input network (E^n(R) feature)"
                                         : "ep_step: the learned push in the Duffing field needs "
                                           "a 5-input network");
    ep_status s = prepare_inference(c, dt, eps);
    if (s != EP_OK) return s;
    if ((s = ensure_queue(c)) != EP_OK) return s;
    if (vp && (s = c->field_valid ? ensure_potential(c) : refresh_field(c)) != EP_OK) return s;
    const int K = (int)c->fallback_K;
    const int Kb = vp ? 0 : base_substeps(c);   // base push (Duffing networks only)
    const double dphi = fmod(dt / eps, kTwoPi);
    size_t chunk = kTableEntries / (size_t)(Kb > K ? Kb : K);
    if (chunk < 1) chunk = 1;
    if ((s = ensure_tables(c, chunk * (size_t)K, chunk)) != EP_OK) return s;
    if (Kb > 0 && (s = ensure_base(c, chunk * (size_t)Kb, chunk, true)) != EP_OK) return s;
    const MeshArgs ma = c->mesh();
    uint64_t done = 0;
    while (done < n_steps) {
        const uint64_t rem = n_steps - done;
        const int S = (int)(rem < chunk ? rem : chunk);
        HIPCHK(c, launch_phase_table(c->stream, c->tab, c->phase, dphi, dt / ((double)K * eps),
                                     dt / K, K, S));
        if (Kb > 0)
            HIPCHK(c, launch_phase_table(c->stream, L.btab, c->phase, dphi,
                                         dt / ((double)Kb * eps), dt / Kb, Kb, S));
        for (int j = 0; j < S; ++j) {
            const double p0 = fmod(c->phase + (double)j * dphi, kTwoPi);
            const double p1 = fmod(c->phase + (double)(j + 1) * dphi, kTwoPi);
            const double2 rot0 = make_double2(cos(p0), sin(p0));
            const double2 rot1 = make_double2(cos(p1), sin(p1));
            const double4 *sub = c->tab.sub + (size_t)j * K;
            const FallbackProjection fproj{L.project ? 1 : 0, rot0, rot1, 0.5 / eps};
            HIPCHK(c, hipMemsetAsync(L.d_qcount, 0, sizeof(unsigned), c->stream));
            if (vp) {
                HIPCHK(c, timed_launch(c, "mlp_push", [&] {
                           return launch_mlp_push_poisson(c->stream, c->zR, c->zV, (int64_t)c->n,
                                                          L.infer, rot0, rot1, eps, c->drift_tol,
                                                          L.d_qcount, L.d_queue, ma,
                                                          c->cfg.r_max, c->n_cu);
                       }));
                HIPCHK(c, timed_launch(c, "fallback_push", [&] {
                           return launch_fallback_poisson(c->stream, c->zR, c->zV, L.d_queue,
                                                          L.d_qcount, sub, K, rot1, ma,
                                                          c->cfg.r_max, fproj, L.d_total,
                                                          c->n_cu);
                       }));
                // the next learned step checks energies with this field's potential
                if (ep_status s2 = solve_mesh(c, ma, true); s2 != EP_OK) return s2;
            } else {
                if (Kb > 0)
                    HIPCHK(c, timed_launch(c, "base_push", [&] {
                               return launch_base_push_duffing(c->stream, c->zR, c->zV, L.d_cR,
                                                               L.d_cV, (int64_t)c->n,
                                                               L.btab.sub + (size_t)j * Kb, Kb);
                           }));
                HIPCHK(c, timed_launch(c, "mlp_push", [&] {
                           return launch_mlp_push_duffing(
                               c->stream, c->zR, c->zV, Kb > 0 ? L.d_cR : nullptr,
                               Kb > 0 ? L.d_cV : nullptr, (int64_t)c->n, L.infer, rot0, rot1, eps,
                               c->drift_tol, L.d_qcount, L.d_queue, c->n_cu);
                       }));
                HIPCHK(c, timed_launch(c, "fallback_push", [&] {
                           return launch_fallback_duffing(c->stream, c->zR, c->zV, L.d_queue,
                                                          L.d_qcount, sub, K, fproj, L.d_total,
                                                          c->n_cu);
                       }));
            }
        }
        c->phase = fmod(c->phase + (double)S * dphi, kTwoPi);
        c->t += (double)S * dt;
        c->n_steps += (uint64_t)S;
        done += (uint64_t)S;
    }
    c->field_valid = vp;
    return EP_OK;
}

}  // namespace etd

extern "C" {

ep_status ep_mlp_set_precision(ep_ctx *c, int32_t precision)
{
    if (!c) return EP_EINVAL;
    if (precision != EP_MLP_BF16 && precision != EP_MLP_FP16)
        return c->fail(EP_EINVAL, "ep_mlp_set_precision: unknown precision %d", (int)precision);
    if (c->mlp.precision != precision) c->mlp.packed = false;
    c->mlp.precision = precision;
    return EP_OK;
}

ep_status ep_mlp_set_projection(ep_ctx *c, int32_t on)
{
    if (!c) return EP_EINVAL;
    if (on != 0 && on != 1)
        return c->fail(EP_EINVAL, "ep_mlp_set_projection: on must be 0 or 1, not %d", (int)on);
    if (c->mlp.project != (on == 1)) c->mlp.packed = false;
    c->mlp.project = on == 1;
    return EP_OK;
}

ep_status ep_mlp_set_weights(ep_ctx *c, const float *params, uint32_t n_params, const double *norm)
{
    if (!c) return EP_EINVAL;
    int n_in = 0;
    if (n_params == (uint32_t)mlp_n_params(5)) n_in = 5;
    if (n_params == (uint32_t)mlp_n_params(6)) n_in = 6;
    if (!params || !norm || n_in == 0)
        return c->fail(EP_EINVAL, "ep_mlp_set_weights: need %d (5 inputs) or %d (6 inputs) "
                                  "parameters and %d normalisation values",
                       mlp_n_params(5), mlp_n_params(6), kNormLen);
    if (!(norm[0] > 0.0) || !(norm[1] > 0.0) || !(norm[2] > 0.0))
        return c->fail(EP_EINVAL, "ep_mlp_set_weights: feature scales must be positive");
    if (norm[7] != 0.0 && norm[7] != 1.0)
        return c->fail(EP_EINVAL, "ep_mlp_set_weights: norm[7] (output map) must be 0 or 1");
    if (!(norm[8] >= 0.0 && norm[8] <= (double)kMaxBaseK) || norm[8] != floor(norm[8]))
        return c->fail(EP_EINVAL, "ep_mlp_set_weights: norm[8] (base push substeps) must be a "
                                  "whole number in [0, %u]", kMaxBaseK);
    if (norm[8] > 0.0 && n_in != 5)
        return c->fail(EP_EINVAL, "ep_mlp_set_weights: a base push (norm[8] > 0) is supported "
                                  "for the Duffing field's 5-input network only");
    DeviceGuard guard(c->device);
    ep_status s = ensure_mlp_buffers(c, n_in);
    if (s != EP_OK) return s;
    Learned &L = c->mlp;
    L.params.assign(params, params + n_params);
    for (int i = 0; i < kNormLen; ++i) L.norm[i] = norm[i];
    HIPCHK(c, copy_sync(c, L.d_params, params, n_params * sizeof(float), hipMemcpyHostToDevice));
    L.packed = false;
    return EP_OK;
}

ep_status ep_mlp_get_weights(ep_ctx *c, float *params, uint32_t n_params, double *norm)
{
    if (!c) return EP_EINVAL;
    if (c->mlp.n_in == 0) return c->fail(EP_ENOTRAINED, "ep_mlp_get_weights: no network loaded");
    if (!params || !norm || n_params != (uint32_t)c->mlp.params.size())
        return c->fail(EP_EINVAL, "ep_mlp_get_weights: n_params must be %zu",
                       c->mlp.params.size());
    memcpy(params, c->mlp.params.data(), n_params * sizeof(float));
    for (int i = 0; i < kNormLen; ++i) norm[i] = c->mlp.norm[i];
    return EP_OK;
}

ep_status ep_mlp_labels(ep_ctx *c, double dt, double eps, uint32_t K, const double *R,
                        const double *V, uint64_t n, float *delta, float *kappa)
{
    if (!c) return EP_EINVAL;
    if (!(dt > 0.0) || !(eps > 0.0) || K == 0 || (n > 0 && (!R || !V || !delta || !kappa)))
        return c->fail(EP_EINVAL, "ep_mlp_labels: need dt > 0, eps > 0, K >= 1");
    if (n == 0) return EP_OK;
    DeviceGuard guard(c->device);
    DevBuf<float> dX, dY;
    HIPCHK(c, dalloc(&dX.p, (size_t)n * 5));
    HIPCHK(c, dalloc(&dY.p, (size_t)n * 2));
    ep_status s = make_labels(c, dt, eps, K, base_substeps(c), 1.0, 0, R, V, n, dX.p, dY.p);
    if (s != EP_OK) return s;
    std::vector<float> Y((size_t)n * 2);
    HIPCHK(c, copy_sync(c, Y.data(), dY.p, Y.size() * sizeof(float), hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < n; ++i) {
        delta[i] = Y[2 * i];
        kappa[i] = Y[2 * i + 1];
    }
    return EP_OK;
}

ep_status ep_mlp_grad(ep_ctx *c, const float *X, const float *Y, uint32_t batch, float *grad,
                      double *loss)
{
    if (!c) return EP_EINVAL;
    Learned &L = c->mlp;
    if (L.n_in == 0) return c->fail(EP_ENOTRAINED, "ep_mlp_grad: no network loaded");
    if (!X || !Y || !grad || batch == 0)
        return c->fail(EP_EINVAL, "ep_mlp_grad: need a batch >= 1 and output arrays");
    DeviceGuard guard(c->device);
    const int np = mlp_n_params(L.n_in);
    const int tiles = (int)((batch + 63) / 64);
    DevBuf<float> dX, dY, gpart, lpart, dloss;
    HIPCHK(c, dalloc(&dX.p, (size_t)batch * L.n_in));
    HIPCHK(c, dalloc(&dY.p, (size_t)batch * 2));
    HIPCHK(c, dalloc(&gpart.p, (size_t)tiles * np));
    HIPCHK(c, dalloc(&lpart.p, (size_t)tiles));
    HIPCHK(c, dalloc(&dloss.p, (size_t)1));
    HIPCHK(c, copy_sync(c, dX.p, X, (size_t)batch * L.n_in * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(c, copy_sync(c, dY.p, Y, (size_t)batch * 2 * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(c, setup_train_lds(L.n_in));
    const float nf[4] = {(float)L.norm[3], (float)(1.0 / L.norm[4]), (float)L.norm[5],
                         (float)(1.0 / L.norm[6])};
    HIPCHK(c, launch_mlp_grad(c->stream, L.n_in, L.d_params, dX.p, dY.p, 0, (int)batch, nf,
                              gpart.p, lpart.p, L.d_grad, dloss.p));
    float lo = 0.f;
    HIPCHK(c, hipMemcpyAsync(grad, L.d_grad, (size_t)np * sizeof(float), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(&lo, dloss.p, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (loss) *loss = lo;
    return EP_OK;
}

ep_status ep_mlp_collect(ep_ctx *c, double dt, double eps, uint32_t K, uint64_t first,
                         uint64_t stride, int32_t reset, uint64_t *n_total)
{
    if (!c) return EP_EINVAL;
    Learned &L = c->mlp;
    if (L.n_in != 6)
        return c->fail(EP_ENOTRAINED, "ep_mlp_collect: load a 6-input network first (its feature "
                                      "scales normalise the samples)");
    if (!(dt > 0.0) || !(eps > 0.0) || !isfinite(dt) || !isfinite(eps) || K == 0 || stride == 0)
        return c->fail(EP_EINVAL, "ep_mlp_collect: need dt > 0, eps > 0, K >= 1, stride >= 1");
    if (c->w <= 0.0) return c->fail(EP_ESTATE, "ep_mlp_collect: no particles loaded");
    DeviceGuard guard(c->device);
    if (reset) L.t_n = 0;
    const uint64_t count = first < c->n ? (c->n - first + stride - 1) / stride : 0;
    if (count) {
        ep_status s;
        if (!c->field_valid && (s = refresh_field(c)) != EP_OK) return s;
        if (L.t_n + count > L.t_cap) {
            uint64_t cap = L.t_cap * 2;
            if (cap < L.t_n + count) cap = L.t_n + count;
            float *nx = nullptr, *ny = nullptr;
            HIPCHK(c, dalloc(&nx, (size_t)cap * 6));
            if (dalloc(&ny, (size_t)cap * 2) != hipSuccess) {
                (void)hipFree(nx);
                return c->fail(EP_ENOMEM, "ep_mlp_collect: no device memory for %llu samples",
                               (unsigned long long)cap);
            }
            hipError_t e = hipSuccess;
            if (L.t_n) {
                e = hipMemcpyAsync(nx, L.d_tx, L.t_n * 6 * sizeof(float), hipMemcpyDeviceToDevice,
                                   c->stream);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(ny, L.d_ty, L.t_n * 2 * sizeof(float),
                                       hipMemcpyDeviceToDevice, c->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            }
            if (e != hipSuccess) {
                (void)hipFree(nx);
                (void)hipFree(ny);
                return c->hipfail("ep_mlp_collect: grow the sample buffers", e);
            }
            if (L.d_tx) (void)hipFree(L.d_tx);
            if (L.d_ty) (void)hipFree(L.d_ty);
            L.d_tx = nx;
            L.d_ty = ny;
            L.t_cap = cap;
        }
        if ((s = ensure_tables(c, K, 1)) != EP_OK) return s;
        const double th = dt / eps, phi = fmod(th, kTwoPi);
        HIPCHK(c, launch_phase_table(c->stream, c->tab, 0.0, phi, th / K, dt / K, (int)K, 1));
        HIPCHK(c, launch_gen_labels_poisson(
                      c->stream, c->zR, c->zV, (int64_t)first, (int64_t)stride, (int64_t)count,
                      make_double2(cos(c->phase), sin(c->phase)), c->mesh(), c->tab.sub, (int)K,
                      (float)(1.0 / L.norm[0]), (float)cos(phi), (float)sin(phi),
                      (float)(th / L.norm[1]), (float)(1.0 / L.norm[2]), L.norm[7] == 1.0,
                      L.d_tx + L.t_n * 6,
                      L.d_ty + L.t_n * 2));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        L.t_n += count;
    }
    if (n_total) *n_total = L.t_n;
    return EP_OK;
}

ep_status ep_mlp_get_samples(ep_ctx *c, uint64_t first, uint64_t count, float *X, float *Y)
{
    if (!c) return EP_EINVAL;
    Learned &L = c->mlp;
    if (first > L.t_n || count > L.t_n - first || (count && (!X || !Y)))
        return c->fail(EP_EINVAL, "ep_mlp_get_samples: rows [%llu, %llu) outside the %llu "
                                  "collected samples",
                       (unsigned long long)first, (unsigned long long)(first + count),
                       (unsigned long long)L.t_n);
    if (count == 0) return EP_OK;
    DeviceGuard guard(c->device);
    HIPCHK(c, copy_sync(c, X, L.d_tx + first * 6, count * 6 * sizeof(float), hipMemcpyDeviceToHost));
    HIPCHK(c, copy_sync(c, Y, L.d_ty + first * 2, count * 2 * sizeof(float), hipMemcpyDeviceToHost));
    return EP_OK;
}

ep_status ep_mlp_train(ep_ctx *c, const ep_train_cfg *cfg, const double *R, const double *V,
                       uint64_t n, ep_train_report *rep)
{
    if (!c) return EP_EINVAL;
    Learned &L = c->mlp;
    if (L.n_in == 0)
        return c->fail(EP_ENOTRAINED, "ep_mlp_train: load initial weights first");
    const bool vp = cfg && cfg->field == EP_FIELD_POISSON;
    if (vp) n = L.t_n;
    if (!cfg || !rep || (cfg->field != EP_FIELD_DUFFING && !vp) || L.n_in != (vp ? 6 : 5) ||
        (!vp && (!R || !V)) || !(cfg->dt > 0.0) || !(cfg->eps > 0.0) ||
        cfg->fine_substeps == 0 || cfg->batch == 0 || cfg->batch % 64 || cfg->batch > n ||
        cfg->epochs == 0 || !(cfg->lr > 0.0) || !(cfg->lr_final >= 0.0) || !(cfg->s_in > 0.0))
        return c->fail(EP_EINVAL, "ep_mlp_train: invalid configuration (Duffing field with a "
                                  "5-input network and given samples, or Poisson field with a "
                                  "6-input network and collected samples; batch a multiple of "
                                  "64 and <= the sample count; positive rates)");
    DeviceGuard guard(c->device);
    const int n_in = L.n_in;
    const int np = mlp_n_params(n_in);
    DevBuf<float> gX, gY, gpart, lpart, dloss;
    const float *dX = L.d_tx, *dY = L.d_ty;
    Events ev;
    hipEvent_t &e0 = ev.e[0], &e1 = ev.e[1], &e2 = ev.e[2];
    for (hipEvent_t &e : ev.e) HIPCHK(c, hipEventCreate(&e));
    HIPCHK(c, hipEventRecord(e0, c->stream));
    if (!vp) {
        HIPCHK(c, dalloc(&gX.p, (size_t)n * 5));
        HIPCHK(c, dalloc(&gY.p, (size_t)n * 2));
        ep_status s = make_labels(c, cfg->dt, cfg->eps, cfg->fine_substeps, base_substeps(c),
                                  cfg->s_in, L.norm[7] == 1.0, R, V, n, gX.p, gY.p);
        if (s != EP_OK) return s;
        dX = gX.p;
        dY = gY.p;
    }
    HIPCHK(c, hipEventRecord(e1, c->stream));

    // normalisation of the labels from their first samples
    const uint64_t ns = n < kNormSamples ? n : kNormSamples;
    std::vector<float> Yh((size_t)ns * 2);
    HIPCHK(c, copy_sync(c, Yh.data(), dY, Yh.size() * sizeof(float), hipMemcpyDeviceToHost));
    double m[2] = {0, 0}, q[2] = {0, 0};
    for (uint64_t i = 0; i < ns; ++i)
        for (int j = 0; j < 2; ++j) m[j] += Yh[2 * i + j];
    for (int j = 0; j < 2; ++j) m[j] /= (double)ns;
    for (uint64_t i = 0; i < ns; ++i)
        for (int j = 0; j < 2; ++j) q[j] += (Yh[2 * i + j] - m[j]) * (Yh[2 * i + j] - m[j]);
    double sd[2];
    for (int j = 0; j < 2; ++j) {
        sd[j] = sqrt(q[j] / (double)ns);
        if (!(sd[j] > 0.0)) sd[j] = 1.0;
    }
    if (!vp) {
        // the Duffing features were just made with these scales
        L.norm[0] = cfg->s_in;
        L.norm[1] = kTimeScale;
        L.norm[2] = 1.0;
    }
    L.norm[3] = m[0];
    L.norm[4] = sd[0];
    L.norm[5] = m[1];
    L.norm[6] = sd[1];
    L.packed = false;
    const float nf[4] = {(float)m[0], (float)(1.0 / sd[0]), (float)m[1], (float)(1.0 / sd[1])};

    const int batch = (int)cfg->batch;
    const int tiles = batch / 64;
    const uint64_t per_epoch = n / (uint64_t)batch;
    const uint64_t T = per_epoch * cfg->epochs;
    HIPCHK(c, dalloc(&gpart.p, (size_t)tiles * np));
    HIPCHK(c, dalloc(&lpart.p, (size_t)tiles));
    HIPCHK(c, dalloc(&dloss.p, (size_t)T));
    HIPCHK(c, hipMemsetAsync(L.d_m, 0, np * sizeof(float), c->stream));
    HIPCHK(c, hipMemsetAsync(L.d_v, 0, np * sizeof(float), c->stream));
    HIPCHK(c, setup_train_lds(n_in));
    for (uint64_t t = 0; t < T; ++t) {
        const uint64_t b = t % per_epoch;
        // Duffing: consecutive i.i.d. samples; collected sets: batch b takes
        // rows b, b + per_epoch, ..., so that each batch spans all snapshots
        const int64_t first = vp ? (int64_t)b : (int64_t)(b * batch);
        const int64_t sstride = vp ? (int64_t)per_epoch : 1;
        const double lr = cfg->lr_final + 0.5 * (cfg->lr - cfg->lr_final) *
                                              (1.0 + cos(3.141592653589793 * (double)t / (double)T));
        const double bc1 = 1.0 / (1.0 - pow(kAdamB1, (double)(t + 1)));
        const double bc2 = 1.0 / (1.0 - pow(kAdamB2, (double)(t + 1)));
        HIPCHK(c, launch_mlp_train_step(c->stream, n_in, L.d_params, L.d_m, L.d_v, dX, dY, first,
                                        sstride, batch, nf, gpart.p, lpart.p, L.d_grad,
                                        dloss.p + t, (float)lr, (float)kAdamB1, (float)kAdamB2,
                                        (float)bc1, (float)bc2, (float)kAdamEps));
    }
    HIPCHK(c, hipEventRecord(e2, c->stream));
    std::vector<float> losses((size_t)T);
    HIPCHK(c, hipMemcpyAsync(losses.data(), dloss.p, T * sizeof(float), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(L.params.data(), L.d_params, np * sizeof(float),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    float ms_label = 0.f, ms_train = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms_label, e0, e1));
    HIPCHK(c, hipEventElapsedTime(&ms_train, e1, e2));
    double lf = 0.0, ll = 0.0;
    for (uint64_t t = 0; t < per_epoch; ++t) {
        lf += losses[t];
        ll += losses[T - per_epoch + t];
    }
    rep->steps = T;
    rep->loss_first = lf / (double)per_epoch;
    rep->loss_last = ll / (double)per_epoch;
    rep->mu_delta = m[0];
    rep->sig_delta = sd[0];
    rep->mu_kappa = m[1];
    rep->sig_kappa = sd[1];
    rep->label_ms = ms_label;
    rep->train_ms = ms_train;
    L.packed = false;
    return EP_OK;
}

}  // extern "C"
