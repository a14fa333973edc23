// HIP kernels of the learned Duhamel corrector (gfx950).
//
// Network 5 (or 6) -> 64 -> 64 -> 2 with the inverse-square-root unit
// act(z) = z / sqrt(1 + z^2).  Its two outputs give the per-step Duhamel term
// of eq. 3.6 in polar form around the exact rotation: a phase advance delta
// and a relative amplitude change kappa, y_{n+1} = (1 + kappa) r(dt/eps + delta)
// y_n.  In the rotating frame z = r(-t/eps) y this is z_{n+1} = (1 + kappa)
// r(delta) z_n.
//
//   gen_labels_duffing_kernel  training pairs: the plain push with K_fine
//                              substeps (FP64 in registers) gives the labels
//                              (around a plain push of K_b substeps, if any)
//   gen_labels_poisson_kernel  the same in a frozen Poisson field, from
//                              collected snapshots of a beam
//   base_push_duffing_kernel   the plain push of K_b substeps whose result the
//                              network corrects (Duffing field, optional)
//   mlp_train_kernel           forward + backward of a 64-sample tile; the
//                              three 64x64x64 products run on BF16 MFMA with
//                              FP32 accumulation (forward split into hi/lo
//                              BF16 halves, three MFMAs, for ~16-bit operands)
//   mlp_grad_reduce_kernel     per-tile gradients summed in a fixed order,
//                              fused with Adam on the FP32 master weights
//   mlp_push_kernel            inference (Duffing or Poisson field, BF16 or
//                              FP16 operands): 64 particles per wave, weights
//                              in LDS, FP64 energy check and optional energy
//                              projection, failing particles appended to a
//                              queue; with the Poisson field, the deposit of
//                              the particles that pass
//   fallback_duffing_kernel    plain push of the queued particles
//   fallback_poisson_kernel    plain push and deposit of the queued particles
//                              in the frozen Poisson field

#include "pic_device.h"

namespace etd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ------------------------------------------------------------ helpers

__device__ __forceinline__ float act(float z) { return z * __frsqrt_rn(fmaf(z, z, 1.f)); }

// act'(z) from h = act(z): (1 - h^2)^(3/2)
__device__ __forceinline__ float act_grad_h(float h)
{
    const float t = fmaf(-h, h, 1.f);
    return t * __fsqrt_rn(t);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two FP32 values -> a packed BF16 pair, round to nearest even (one
// v_cvt_pk_bf16_f32 on gfx950); element 0 in the low half.
__device__ __forceinline__ unsigned pack_bf16x2(float a, float b)
{
    const f32x2 v = {a, b};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}

// Eight FP32 values as a BF16 MFMA operand (hi), and optionally the BF16 of
// their remainders (lo = bf16(a - hi), exact subtraction), so that hi + lo
// carries ~16 significant bits.
template <bool SPLIT>
__device__ __forceinline__ void to_bf16x8(const float (&a)[8], bf16x8 &hi, bf16x8 &lo)
{
    uint4 h, l;
    unsigned *hp = &h.x, *lp = &l.x;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        hp[i] = pack_bf16x2(a[2 * i], a[2 * i + 1]);
        if (SPLIT)
            lp[i] = pack_bf16x2(a[2 * i] - __uint_as_float(hp[i] << 16),
                                a[2 * i + 1] - __uint_as_float(hp[i] & 0xFFFF0000u));
    }
    hi = __builtin_bit_cast(bf16x8, h);
    if (SPLIT) lo = __builtin_bit_cast(bf16x8, l);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 q) { return __builtin_bit_cast(bf16x8, q); }

typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f16x8 as_f16x8(uint4 q) { return __builtin_bit_cast(f16x8, q); }

extern "C" __device__ _Float16 __ocml_rsqrt_f16(_Float16);

// The activation of two pre-activations given as u = z / 64 (FP32), in
// packed FP16: act(z) = z / sqrt(1 + z^2) = u / sqrt(u^2 + 2^-12).  The 1/64
// keeps u^2 finite for |z| < 16320 and 2^-12 a normal FP16 number; the
// inference weights carry the factor.  Inputs are rounded to nearest once;
// the result has ~11 significant bits.
__device__ __forceinline__ f16x2 act_pair(float a, float b)
{
    const f16x2 u = {(_Float16)a, (_Float16)b};
    const f16x2 c = {(_Float16)0x1p-12f, (_Float16)0x1p-12f};
    const f16x2 t = __builtin_elementwise_fma(u, u, c);
    const f16x2 r = {__ocml_rsqrt_f16(t.x), __ocml_rsqrt_f16(t.y)};
    return u * r;
}

// Operand types of the inference MFMAs (32x32x16, FP32 accumulation).
//   FP16: activations in packed FP16 arithmetic, W2 and W3 in FP16 (one
//         MFMA each);
//   BF16: gfx950 has no packed BF16 arithmetic, so the activations run in
//         FP32 and are rounded to BF16; W2 and W3 as split BF16 (hi + lo, two
//         MFMAs, ~16 bits), and the activations into layers 2 and 3 as
//         hi + lo too (a third MFMA, weights hi times activations lo): their
//         8-bit rounding was the largest error term.
// Both take the pre-activations as u = z / 64 (see act_pair).
template <typename T>
struct InferOp;

template <>
struct InferOp<_Float16> {
    typedef f16x8 vec;
    static constexpr bool kSplitW = false;
    static constexpr bool kSplitA3 = false;   // activations into layers 2, 3 as hi + lo
    static __device__ __forceinline__ vec load(uint4 q) { return __builtin_bit_cast(vec, q); }
    static __device__ __forceinline__ f32x16 mma(vec a, vec b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
    // activations of accumulator elements q0 .. q0 + 7
    static __device__ __forceinline__ vec act(const f32x16 &acc, int q0)
    {
        vec v;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const f16x2 h = act_pair(acc[q0 + 2 * i], acc[q0 + 2 * i + 1]);
            v[2 * i] = h.x;
            v[2 * i + 1] = h.y;
        }
        return v;
    }
};

template <>
struct InferOp<__bf16> {
    typedef bf16x8 vec;
    static constexpr bool kSplitW = true;
    static constexpr bool kSplitA3 = true;
    static __device__ __forceinline__ vec load(uint4 q) { return __builtin_bit_cast(vec, q); }
    static __device__ __forceinline__ f32x16 mma(vec a, vec b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ vec act(const f32x16 &acc, int q0)
    {
        uint4 h;
        unsigned *hp = &h.x;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float u0 = acc[q0 + 2 * i], u1 = acc[q0 + 2 * i + 1];
            hp[i] = pack_bf16x2(u0 * __frsqrt_rn(fmaf(u0, u0, 0x1p-12f)),
                                u1 * __frsqrt_rn(fmaf(u1, u1, 0x1p-12f)));
        }
        return __builtin_bit_cast(vec, h);
    }
    // The same activations as hi (the bits of act) and lo = bf16(a - hi).
    static __device__ __forceinline__ vec act_split(const f32x16 &acc, int q0, vec &lo)
    {
        float a[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float u = acc[q0 + i];
            a[i] = u * __frsqrt_rn(fmaf(u, u, 0x1p-12f));
        }
        vec hi;
        to_bf16x8<true>(a, hi, lo);
        return hi;
    }
};

// Wave-level 32x32 tile of a 64x64x64 product from FP32 LDS operands:
//   acc(i, j) += sum_k A(i0 + i, k) B(k, j0 + j),
//   A(i, k) = A[i*ai + k*ak],  B(k, j) = B[k*bk + j*bj].
// MFMA 32x32x16 operand layout: lane l holds rows/cols (l % 32) and the 8
// consecutive k of group (l / 32) of each 16-wide k step; result element q of
// lane l is (i = 8 (q/4) + 4 (l/32) + q%4, j = l % 32).
template <bool SPLIT>
__device__ void mma64_wave(const float *A, int ai, int ak, const float *B, int bk, int bj, int i0,
                           int j0, f32x16 &acc)
{
    const int lane = threadIdx.x & 63;
    const int r = lane & 31, g = lane >> 5;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        float a[8], b[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = kk * 16 + g * 8 + e;
            a[e] = A[(i0 + r) * ai + k * ak];
            b[e] = B[k * bk + (j0 + r) * bj];
        }
        bf16x8 ah, al, bh, bl;
        to_bf16x8<SPLIT>(a, ah, al);
        to_bf16x8<SPLIT>(b, bh, bl);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
        if (SPLIT) {
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
        }
    }
}

__device__ __forceinline__ int tile_row(int q, int g) { return 8 * (q >> 2) + 4 * g + (q & 3); }

// Polar form of a step from z0 to z1 (rotating frame, so the free rotation is
// the identity): delta = angle from z0 to z1 in the direction r advances,
// kappa = |z1| / |z0| - 1; scaled: (|z0| delta, |z1| - |z0|).
__device__ __forceinline__ void polar_label(double zr0, double zv0, double zr, double zv,
                                            int scaled, double &delta, double &kappa)
{
    const double n0 = sqrt(zr0 * zr0 + zv0 * zv0), n1 = sqrt(zr * zr + zv * zv);
    delta = kappa = 0.0;
    if (n0 > 0.0) {
        delta = atan2(zr * zv0 - zv * zr0, zr * zr0 + zv * zv0);
        if (scaled) {
            delta *= n0;
            kappa = n1 - n0;
        } else {
            kappa = n1 / n0 - 1.0;
        }
    }
}

// ------------------------------------------------------------ labels

// K substeps of the plain Duffing push (FP64, rotating frame) from z.
__device__ __forceinline__ void duffing_substeps(const double4 *__restrict__ sub, int K,
                                                 double &zr, double &zv)
{
    double ar = 0.0, av = 0.0;
    for (int k = 0; k < K; ++k) {
        const double4 q = sub[k];
        const double Rm = fma(q.x, zr + ar, q.y * (zv + av));
        const double E = -(Rm * Rm) * Rm;
        ar = fma(-q.z, E, ar);
        av = fma(q.w, E, av);
    }
    zr += ar;
    zv += av;
}

// Training pairs for the Duffing field.  Each sample y = (R, V) is pushed one
// step with the plain scheme (K_fine substeps, FP64) from phase 0; the labels
// are the polar form of the step from its base point: delta = angle from z_b
// to z_fine in the direction r advances, kappa = |z_fine| / |z_b| - 1.  The
// base point is z_n itself (the free rotation, the identity in the rotating
// frame) or, with Kb > 0, the plain push of z_n with Kb substeps (table bsub).
// Features x = (R/s_in, V/s_in, cos phi, sin phi, (dt/eps)/s_t).
__global__ __launch_bounds__(256) void gen_labels_duffing_kernel(
    const float *__restrict__ Rs, const float *__restrict__ Vs, int64_t n,
    const double4 *__restrict__ sub, int K, const double4 *__restrict__ bsub, int Kb,
    float inv_sin, float c_phi, float s_phi, float th_scaled, int scaled, float *__restrict__ X,
    float *__restrict__ Y)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float R = Rs[i], V = Vs[i];
    double zr0 = R, zv0 = V;
    double zr = zr0, zv = zv0;
    duffing_substeps(sub, K, zr, zv);
    if (Kb > 0) duffing_substeps(bsub, Kb, zr0, zv0);
    double delta, kappa;
    polar_label(zr0, zv0, zr, zv, scaled, delta, kappa);
    float *x = X + i * 5;
    x[0] = R * inv_sin;
    x[1] = V * inv_sin;
    x[2] = c_phi;
    x[3] = s_phi;
    x[4] = th_scaled;
    Y[i * 2] = (float)delta;
    Y[i * 2 + 1] = (float)kappa;
}

hipError_t launch_gen_labels_duffing(hipStream_t st, const float *R, const float *V, int64_t n,
                                     const double4 *sub, int K, const double4 *bsub, int Kb,
                                     float inv_sin, float c_phi, float s_phi, float th_scaled,
                                     int scaled, float *X, float *Y)
{
    if (n <= 0) return hipSuccess;
    gen_labels_duffing_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(
        R, V, n, sub, K, bsub, Kb, inv_sin, c_phi, s_phi, th_scaled, scaled, X, Y);
    return hipGetLastError();
}

// Base push of a learned step with a base (Duffing field): the plain push of
// every particle with Kb substeps (FP64, table sub of this step), from z into
// the base arrays c, rounded to FP32 once.  The network then corrects c.
__global__ __launch_bounds__(256) void base_push_duffing_kernel(
    const float *__restrict__ zR, const float *__restrict__ zV, float *__restrict__ cR,
    float *__restrict__ cV, int64_t n, const double4 *__restrict__ sub, int Kb)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double zr = zR[i], zv = zV[i];
    duffing_substeps(sub, Kb, zr, zv);
    cR[i] = (float)zr;
    cV[i] = (float)zv;
}

hipError_t launch_base_push_duffing(hipStream_t st, const float *zR, const float *zV, float *cR,
                                    float *cV, int64_t n, const double4 *sub, int Kb)
{
    if (n <= 0) return hipSuccess;
    const int block = 256;
    return dispatch(base_push_duffing_kernel, dim3((unsigned)((n + block - 1) / block)),
                    dim3(block), 0, st, zR, zV, cR, cV, n, sub, Kb);
}

// Training pairs from the self-consistent beam: sample j is particle
// first + j * stride of the context at time t_n (lab frame y_n = r(Phi_n) z).
// Its label is the plain push with K_fine substeps (FP64) in the frozen field
// E^n of the current mesh, started from phase 0 (the frozen-field step is
// autonomous, so the map does not depend on Phi_n).  Features as for the
// Duffing field plus E^n(R_n) / s_E, gathered as the inference kernel does.
__global__ __launch_bounds__(256) void gen_labels_poisson_kernel(
    const float *__restrict__ zR, const float *__restrict__ zV, int64_t first, int64_t stride,
    int64_t count, double2 rot0, MeshView m, const double *__restrict__ fscal,
    const double4 *__restrict__ sub, int K, float inv_sin, float c_phi, float s_phi,
    float th_scaled, float inv_sE, int scaled, float *__restrict__ X, float *__restrict__ Y)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= count) return;
    m.Qb = fscal[kQb];
    const int64_t i = first + j * stride;
    const double zr_ = zR[i], zv_ = zV[i];
    const double zr0 = fma(rot0.x, zr_, rot0.y * zv_);
    const double zv0 = fma(-rot0.y, zr_, rot0.x * zv_);
    const double E0 = gather(m, zr0);
    double zr = zr0, zv = zv0;
    {
        double a[1] = {zr}, b[1] = {zv};
        if (fma(zr, zr, zv * zv) < on_mesh_limit2(m, sub, K, fscal[kEmax]))
            push_group<1, true>(m, sub, K, a, b);
        else
            push_group<1>(m, sub, K, a, b);
        zr = a[0];
        zv = b[0];
    }
    double delta, kappa;
    polar_label(zr0, zv0, zr, zv, scaled, delta, kappa);
    float *x = X + j * 6;
    x[0] = (float)zr0 * inv_sin;
    x[1] = (float)zv0 * inv_sin;
    x[2] = c_phi;
    x[3] = s_phi;
    x[4] = th_scaled;
    x[5] = (float)E0 * inv_sE;
    Y[j * 2] = (float)delta;
    Y[j * 2 + 1] = (float)kappa;
}

hipError_t launch_gen_labels_poisson(hipStream_t st, const float *zR, const float *zV,
                                     int64_t first, int64_t stride, int64_t count, double2 rot0,
                                     const MeshArgs &ma, const double4 *sub, int K, float inv_sin,
                                     float c_phi, float s_phi, float th_scaled, float inv_sE,
                                     int scaled, float *X, float *Y)
{
    if (count <= 0) return hipSuccess;
    MeshView m;
    m.Et = ma.etab;
    m.H = nullptr;
    m.inv_hr = 1.0 / ma.hr;
    m.half = 0.5 * (double)ma.nr;
    m.c = ma.nr >> 1;
    m.Qb = 0.0;   // read on the device from fscal
    gen_labels_poisson_kernel<<<dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st>>>(
        zR, zV, first, stride, count, rot0, m, (const double *)ma.fscal, sub, K, inv_sin, c_phi, s_phi,
        th_scaled, inv_sE, scaled, X, Y);
    return hipGetLastError();
}

// ------------------------------------------------------------ training

constexpr int kTile = 64;   // samples per training workgroup
constexpr int kLd = kH + 1; // LDS row stride of the 64x64 matrices (no bank conflicts)

// A tile is one workgroup of 16 waves.  The three products run on waves 0-3
// (one 32 x 32 block each; in the backward pass dW2 on waves 0-3 and dH1 on
// waves 4-7 at once); every other phase is spread over all 1024 threads, so
// that no wave walks a long dependent chain (one wave per SIMD, as with four
// waves, left the tile bound by the latency of its instructions).
constexpr int kTrainBlock = 1024, kTrainWaves = kTrainBlock / 64;
// sums over the 64 samples of a tile: kSampleParts partial sums of 4 samples
// (db2, dW1, db1) or kOutParts of 8 (dW3), added in a fixed pairwise tree
constexpr int kSampleParts = 16, kOutParts = 8;
// partial sums of the layer-1 gradients: [16 sample parts][64 units][n_in + 1]
constexpr int kPartStride = 8;

static size_t train_lds_floats(int n_in)
{
    return (size_t)mlp_n_params(n_in) + kTile * n_in + kTile * 2 + 5 * kTile * kLd + kTile * 2 +
           kOutParts * kOut * kH + kSampleParts * kH + kSampleParts * kH * kPartStride +
           kTrainWaves;
}

// Sum of n = 2^m values v[0], v[stride], ... in a fixed pairwise tree.
template <int N>
__device__ __forceinline__ float tree_sum(const float *v, int stride)
{
    if constexpr (N == 1) {
        return v[0];
    } else {
        return tree_sum<N / 2>(v, stride) + tree_sum<N / 2>(v + (N / 2) * stride, stride);
    }
}

// Forward and backward of the MSE loss over one tile of 64 samples: sample s
// of the batch is row first + s * sstride of X and Y, samples at or beyond
// `batch` masked out.  Labels are
// normalised on load, Yn = (Y - mu) * inv_sig.  Writes this tile's gradient
// (flat parameter order) to gpart[tile] and its sum of squared errors to
// lpart[tile]; the loss is the mean over the batch and both outputs.
// The three 64 x 64 x 64 products run on MFMA; every other sum over the 64
// samples or units is split into partial sums of 4 or 8 terms that are
// combined in a fixed order, so that the results do not depend on
// scheduling.
template <int NIN>
__global__ __launch_bounds__(kTrainBlock) void mlp_train_kernel(
    const float *__restrict__ params, const float *__restrict__ X, const float *__restrict__ Y,
    int64_t first, int64_t sstride, int batch, float mu_d, float is_d, float mu_k, float is_k,
    float *__restrict__ gpart, float *__restrict__ lpart)
{
    constexpr int NP = kH * NIN + kH + kH * kH + kH + kOut * kH + kOut;
    constexpr int oW1 = 0, ob1 = kH * NIN, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH,
                  ob3 = oW3 + kOut * kH;
    static_assert(NIN + 1 <= kPartStride, "layer-1 partial sums fit their stride");
    static_assert(kTile * (NIN + 2) <= kTrainBlock, "features and labels: one load per thread");
    static_assert(kTile / kSampleParts == 4 && kTile / kOutParts == 8, "partial-sum sizes");
    extern __shared__ __align__(16) float sm[];
    float *sP = sm;                     // parameters (flat)
    float *sX = sP + NP;                // [64][NIN]
    float *sY = sX + kTile * NIN;       // [64][2]
    float *sW2 = sY + kTile * 2;        // [64][kLd] padded copy of W2[u][k]
    float *sH1 = sW2 + kH * kLd;        // [64 samples][kLd]
    float *sH2 = sH1 + kTile * kLd;
    float *sG = sH2 + kTile * kLd;      // dZ2
    float *sD = sG + kTile * kLd;       // dZ1
    float *sdO = sD + kTile * kLd;      // [64][2]
    // partial sums, one region per use: dW3 [8][128], db2 [16][64], dW1 and
    // db1 [16][64][kPartStride]
    float *sQ3 = sdO + kTile * 2;
    float *sQ2 = sQ3 + kOutParts * kOut * kH;
    float *sQ1 = sQ2 + kSampleParts * kH;
    float *sL = sQ1 + kSampleParts * kH * kPartStride;   // [16] loss of each wave

    const int tid = threadIdx.x, nt = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63, r = lane & 31, g = lane >> 5;
    const int s_base = blockIdx.x * kTile;
    float *gp = gpart + (size_t)blockIdx.x * NP;

    // Parameters, features and labels: every global load of the thread is
    // issued before the first LDS store, so their latencies overlap (the
    // parameters as float4; the host buffer is 16-byte aligned).
    {
        constexpr int NP4 = NP / 4, kPer = (NP4 + kTrainBlock - 1) / kTrainBlock;
        const float4 *p4 = reinterpret_cast<const float4 *>(params);
        float4 buf[kPer];
        // unconditional loads (past the end: the last group again), so that
        // buf stays in registers
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int i = tid + j * kTrainBlock;
            buf[j] = p4[i < NP4 ? i : NP4 - 1];
        }
        const int it = 4 * NP4 + tid;
        const float ptail = it < NP ? params[it] : 0.f;
        // one unconditional load: an element of X or Y, or, past the tile's
        // samples, the batch's first sample again, replaced by 0
        float xy;
        {
            const int i = tid;
            const bool isx = i < kTile * NIN;
            const int k = i - kTile * NIN;
            const int s = isx ? i / NIN : k >> 1;
            const bool ok = (isx || k < kTile * 2) && s_base + s < batch;
            const int64_t row = first + (ok ? (int64_t)(s_base + s) * sstride : 0);
            const float *src = isx ? X + row * NIN + (ok ? i - s * NIN : 0)
                                   : Y + row * 2 + (ok ? (k & 1) : 0);
            const float v = *src;
            xy = ok ? v : 0.f;
        }
        // unconditional stores too (past the end: the last group's own value
        // again), so that loads and stores sit in one block and the loads
        // issue together
        float4 *s4 = reinterpret_cast<float4 *>(sP);
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int i = tid + j * kTrainBlock;
            s4[i < NP4 ? i : NP4 - 1] = buf[j];
        }
        if (it < NP) sP[it] = ptail;
        if (tid < kTile * NIN) {
            sX[tid] = xy;
        } else if (tid < kTile * (NIN + 2)) {
            const int k = tid - kTile * NIN;
            sY[k] = (k & 1) ? (xy - mu_k) * is_k : (xy - mu_d) * is_d;
        }
    }
    __syncthreads();
    for (int i = tid; i < kH * kH; i += nt) sW2[(i >> 6) * kLd + (i & 63)] = sP[oW2 + i];
    __syncthreads();

    // layer 1 (VALU): H1[s][u] = act(b1[u] + sum_f W1[u][f] X[s][f])
    for (int i = tid; i < kTile * kH; i += nt) {
        const int s = i >> 6, u = i & 63;
        float z = sP[ob1 + u];
#pragma unroll
        for (int f = 0; f < NIN; ++f) z = fmaf(sP[oW1 + u * NIN + f], sX[s * NIN + f], z);
        sH1[s * kLd + u] = act(z);
    }
    __syncthreads();

    // layer 2 (MFMA, split BF16, waves 0-3): Z2[s][u] = sum_k H1[s][k] W2[u][k]
    const int blk = wave & 3;
    const int i0 = (blk >> 1) * 32, j0 = (blk & 1) * 32;
    if (wave < 4) {
        f32x16 acc = {};
        mma64_wave<true>(sH1, kLd, 1, sW2, 1, kLd, i0, j0, acc);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int s = i0 + tile_row(q, g), u = j0 + r;
            sH2[s * kLd + u] = act(acc[q] + sP[ob2 + u]);
        }
    }
    __syncthreads();

    // layer 3 (VALU), loss and dO = d loss / d O.  Sample s = tid / 16; its
    // 16 threads (lanes of one wave) sum 4 hidden units each.
    {
        const int s = tid >> 4, qu = tid & 15;
        float o0 = 0.f, o1 = 0.f;
#pragma unroll
        for (int u = 4 * qu; u < 4 * qu + 4; ++u) {
            const float h = sH2[s * kLd + u];
            o0 = fmaf(sP[oW3 + u], h, o0);
            o1 = fmaf(sP[oW3 + kH + u], h, o1);
        }
#pragma unroll
        for (int m = 1; m < 16; m <<= 1) {
            o0 += __shfl_xor(o0, m, 64);
            o1 += __shfl_xor(o1, m, 64);
        }
        const bool valid = s_base + s < batch;
        const float d0 = valid ? (o0 + sP[ob3]) - sY[2 * s] : 0.f;
        const float d1 = valid ? (o1 + sP[ob3 + 1]) - sY[2 * s + 1] : 0.f;
        if (qu == 0) {
            sdO[2 * s] = 2.f * d0 / (float)(batch * 2);
            sdO[2 * s + 1] = 2.f * d1 / (float)(batch * 2);
        }
        const float l = wave_sum(qu == 0 ? fmaf(d0, d0, d1 * d1) : 0.f);
        if (lane == 0) sL[wave] = l;
    }
    __syncthreads();
    if (tid == 0) lpart[blockIdx.x] = tree_sum<kTrainWaves>(sL, 1);
    // dW3[m][u] = sum_s dO[s][m] H2[s][u]: thread (m, u) of each eighth of
    // the samples
    {
        const int o = tid & 127, m = o >> 6, u = o & 63, part = tid >> 7;
        float a = 0.f;
#pragma unroll
        for (int s = 8 * part; s < 8 * part + 8; ++s) a = fmaf(sdO[s * 2 + m], sH2[s * kLd + u], a);
        sQ3[part * 128 + o] = a;
    }
    // db3: wave 0, one sample per lane
    if (wave == 0) {
        const float b0 = wave_sum(sdO[2 * lane]), b1 = wave_sum(sdO[2 * lane + 1]);
        if (lane == 0) {
            gp[ob3] = b0;
            gp[ob3 + 1] = b1;
        }
    }
    // G = dZ2 = (dO W3) * act'(Z2)
    for (int i = tid; i < kTile * kH; i += nt) {
        const int s = i >> 6, u = i & 63;
        const float d = fmaf(sdO[s * 2], sP[oW3 + u], sdO[s * 2 + 1] * sP[oW3 + kH + u]);
        sG[s * kLd + u] = d * act_grad_h(sH2[s * kLd + u]);
    }
    __syncthreads();
    if (tid < kOut * kH) gp[oW3 + tid] = tree_sum<kOutParts>(sQ3 + tid, 128);

    if (wave < 4) {
        // dW2[u][k] = sum_s G[s][u] H1[s][k]   (MFMA)
        f32x16 acc = {};
        mma64_wave<false>(sG, 1, kLd, sH1, kLd, 1, i0, j0, acc);
#pragma unroll
        for (int q = 0; q < 16; ++q) gp[oW2 + (i0 + tile_row(q, g)) * kH + j0 + r] = acc[q];
    } else if (wave < 8) {
        // dH1[s][k] = sum_u G[s][u] W2[u][k]   (MFMA), D = dZ1 = dH1 * act'(Z1)
        f32x16 acc = {};
        mma64_wave<false>(sG, kLd, 1, sW2, kLd, 1, i0, j0, acc);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int s = i0 + tile_row(q, g), k = j0 + r;
            sD[s * kLd + k] = acc[q] * act_grad_h(sH1[s * kLd + k]);
        }
    }
    // db2 partials: unit u = tid % 64, samples of part tid / 64
    {
        const int u = tid & 63, part = tid >> 6;
        float a = 0.f;
#pragma unroll
        for (int s = 4 * part; s < 4 * part + 4; ++s) a += sG[s * kLd + u];
        sQ2[part * kH + u] = a;
    }
    __syncthreads();
    if (tid < kH) gp[ob2 + tid] = tree_sum<kSampleParts>(sQ2 + tid, kH);
    // dW1[u][f] = sum_s D[s][u] X[s][f], db1[u] = sum_s D[s][u]: unit u =
    // tid % 64, samples of part tid / 64, all n_in + 1 sums at once
    {
        const int u = tid & 63, part = tid >> 6;
        float a[NIN + 1];
#pragma unroll
        for (int f = 0; f <= NIN; ++f) a[f] = 0.f;
#pragma unroll
        for (int s = 4 * part; s < 4 * part + 4; ++s) {
            const float d = sD[s * kLd + u];
#pragma unroll
            for (int f = 0; f < NIN; ++f) a[f] = fmaf(d, sX[s * NIN + f], a[f]);
            a[NIN] += d;
        }
#pragma unroll
        for (int f = 0; f <= NIN; ++f) sQ1[(part * kH + u) * kPartStride + f] = a[f];
    }
    __syncthreads();
    for (int i = tid; i < kH * (NIN + 1); i += nt) {
        const int u = i / (NIN + 1), f = i - u * (NIN + 1);
        const float v = tree_sum<kSampleParts>(sQ1 + u * kPartStride + f, kH * kPartStride);
        if (f < NIN)
            gp[oW1 + u * NIN + f] = v;
        else
            gp[ob1 + u] = v;
    }
}

// grad[p] = sum over the per-tile gradients, loss = sum of lpart / (batch * 2).
// A workgroup of 256 threads takes 16 parameters; the 16 threads of a
// parameter sum the tiles t = c, c + 16, ... (c = 0..15), and the 16 partial
// sums are added pairwise in a fixed tree, so the result is reproducible.
// With ADAM the update of Adam (Kingma & Ba; bias corrections
// bc1 = 1/(1 - b1^t), bc2 = 1/(1 - b2^t)) is applied to the parameters too.
struct AdamArgs {
    float *p, *m, *v;
    float lr, b1, b2, bc1, bc2, eps;
};

constexpr int kRedParams = 16, kRedChunks = 16;

template <bool ADAM>
__global__ __launch_bounds__(kRedParams * kRedChunks) void mlp_grad_reduce_kernel(
    const float *__restrict__ gpart, const float *__restrict__ lpart, int tiles, int np, int batch,
    float *__restrict__ grad, float *__restrict__ loss, AdamArgs ad)
{
    __shared__ float part[kRedChunks][kRedParams];
    __shared__ double lw[4];
    const int tid = threadIdx.x, pl = tid % kRedParams, c = tid / kRedParams;
    const int p = blockIdx.x * kRedParams + pl;
    // the Adam state of the parameter, read before the sum so that its
    // latency overlaps the partial sums' (clamped, unconditional loads)
    float m0 = 0.f, v0 = 0.f, p0 = 0.f;
    if (ADAM) {
        const int pc = p < np ? p : np - 1;
        m0 = ad.m[pc];
        v0 = ad.v[pc];
        p0 = ad.p[pc];
    }
    // rows c, c + 16, c + 32, ... summed in that order; four loads in flight
    float a = 0.f;
    if (p < np) {
        int t = c;
        for (; t + 3 * kRedChunks < tiles; t += 4 * kRedChunks) {
            const float g0 = gpart[(size_t)t * np + p];
            const float g1 = gpart[(size_t)(t + kRedChunks) * np + p];
            const float g2 = gpart[(size_t)(t + 2 * kRedChunks) * np + p];
            const float g3 = gpart[(size_t)(t + 3 * kRedChunks) * np + p];
            a += g0;
            a += g1;
            a += g2;
            a += g3;
        }
        for (; t < tiles; t += kRedChunks) a += gpart[(size_t)t * np + p];
    }
    part[c][pl] = a;
    __syncthreads();
#pragma unroll
    for (int w = kRedChunks / 2; w > 0; w >>= 1) {
        if (c < w) part[c][pl] = part[c][pl] + part[c + w][pl];
        __syncthreads();
    }
    if (c == 0 && p < np) {
        const float gi = part[0][pl];
        grad[p] = gi;
        if (ADAM) {
            const float mi = fmaf(ad.b1, m0, (1.f - ad.b1) * gi);
            const float vi = fmaf(ad.b2, v0, (1.f - ad.b2) * gi * gi);
            ad.m[p] = mi;
            ad.v[p] = vi;
            ad.p[p] = p0 - ad.lr * (mi * ad.bc1) / (__fsqrt_rn(vi * ad.bc2) + ad.eps);
        }
    }
    if (blockIdx.x == 0) {
        double l = 0.0;
        for (int t = tid; t < tiles; t += blockDim.x) l += lpart[t];
        l = wave_sum(l);
        if ((tid & 63) == 0) lw[tid >> 6] = l;
        __syncthreads();
        if (tid == 0) *loss = (float)(((lw[0] + lw[1]) + (lw[2] + lw[3])) / (double)(batch * 2));
    }
}

hipError_t setup_train_lds(int n_in)
{
    const int lds = (int)(train_lds_floats(n_in) * sizeof(float));
    if (n_in == 5)
        return raise_dynamic_lds(reinterpret_cast<const void *>(&mlp_train_kernel<5>), lds);
    return raise_dynamic_lds(reinterpret_cast<const void *>(&mlp_train_kernel<6>), lds);
}

static hipError_t launch_train_tiles(hipStream_t st, int n_in, const float *params,
                                     const float *X, const float *Y, int64_t first,
                                     int64_t sstride, int batch, const float norm[4],
                                     float *gpart, float *lpart)
{
    const int tiles = (batch + kTile - 1) / kTile;
    const size_t lds = train_lds_floats(n_in) * sizeof(float);
    if (n_in == 5)
        mlp_train_kernel<5><<<dim3(tiles), dim3(kTrainBlock), lds, st>>>(
            params, X, Y, first, sstride, batch, norm[0], norm[1], norm[2], norm[3], gpart, lpart);
    else
        mlp_train_kernel<6><<<dim3(tiles), dim3(kTrainBlock), lds, st>>>(
            params, X, Y, first, sstride, batch, norm[0], norm[1], norm[2], norm[3], gpart, lpart);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(hipStream_t st, int n_in, const float *params, const float *X,
                           const float *Y, int64_t first, int batch, const float norm[4],
                           float *gpart, float *lpart, float *grad, float *loss)
{
    hipError_t e =
        launch_train_tiles(st, n_in, params, X, Y, first, 1, batch, norm, gpart, lpart);
    if (e != hipSuccess) return e;
    const int np = mlp_n_params(n_in), tiles = (batch + kTile - 1) / kTile;
    mlp_grad_reduce_kernel<false><<<dim3((np + kRedParams - 1) / kRedParams),
                                    dim3(kRedParams * kRedChunks), 0, st>>>(
        gpart, lpart, tiles, np, batch, grad, loss, AdamArgs{});
    return hipGetLastError();
}

hipError_t launch_mlp_train_step(hipStream_t st, int n_in, float *params, float *m, float *v,
                                 const float *X, const float *Y, int64_t first, int64_t sstride,
                                 int batch, const float norm[4], float *gpart, float *lpart,
                                 float *grad, float *loss, float lr, float b1, float b2, float bc1,
                                 float bc2, float eps)
{
    hipError_t e =
        launch_train_tiles(st, n_in, params, X, Y, first, sstride, batch, norm, gpart, lpart);
    if (e != hipSuccess) return e;
    const int np = mlp_n_params(n_in), tiles = (batch + kTile - 1) / kTile;
    mlp_grad_reduce_kernel<true><<<dim3((np + kRedParams - 1) / kRedParams),
                                   dim3(kRedParams * kRedChunks), 0, st>>>(
        gpart, lpart, tiles, np, batch, grad, loss, AdamArgs{params, m, v, lr, b1, b2, bc1, bc2, eps});
    return hipGetLastError();
}

// ------------------------------------------------------------ inference

constexpr unsigned kWaveQueue = 512;   // LDS fallback-queue entries per wave

// Fallback queue of one wave: a segment of LDS and a wave-uniform fill count.
// A full segment is copied to the global queue with one atomic, so waves
// never wait on each other.
struct WaveQueue {
    unsigned *sq;
    unsigned qn;
};

__device__ __forceinline__ void wave_queue_flush(WaveQueue &q, unsigned *qcount, unsigned *queue,
                                                 int lane)
{
    if (q.qn == 0u) return;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    unsigned base = 0u;
    if (lane == 0) base = atomicAdd(qcount, q.qn);
    base = __shfl(base, 0, 64);
    for (unsigned i = (unsigned)lane; i < q.qn; i += 64u) queue[base + i] = q.sq[i];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    q.qn = 0u;
}

__device__ __forceinline__ void wave_queue_push(WaveQueue &q, bool fail, unsigned p,
                                                unsigned *qcount, unsigned *queue, int lane)
{
    const unsigned long long fm = __ballot(fail);
    if (fm == 0ull) return;
    const unsigned cnt = (unsigned)__popcll(fm);
    if (q.qn + cnt > kWaveQueue) wave_queue_flush(q, qcount, queue, lane);
    if (fail) q.sq[q.qn + (unsigned)__popcll(fm & ((1ull << lane) - 1ull))] = p;
    q.qn += cnt;
}

// Frozen-field potential Psi^n(R) with -dPsi/dR = E^n(R): the exact integral
// of the CIC field from the FP64 node values (piecewise quadratic on each
// cell); outside the mesh Psi(+-r_max) - Qb ln(|R| / r_max).
struct PotView {
    const double *E, *Psi;
    double hr, inv_hr, half, rmax, Qb;
    int c, nr;
};

__device__ __forceinline__ double potential(const PotView &v, double R)
{
    const double x = R * v.inv_hr;
    if (x >= v.half) return v.Psi[v.nr] - v.Qb * log(R / v.rmax);
    if (x < -v.half) return v.Psi[0] - v.Qb * log(-R / v.rmax);
    if (!(x == x)) return x;
    const double fl = floor(x);
    const int m = (int)fl + v.c;
    const double d = (x - fl) * v.hr;
    const double e0 = v.E[m], e1 = v.E[m + 1];
    return v.Psi[m] - fma(e0, d, (e1 - e0) * (d * d) * (0.5 * v.inv_hr));
}

// One Newton step of the radial projection z <- s z onto the energy H0 from
// s = 1 (H1 the energy at z, RdP = R P'(R) at its lab position): the slope
// dH/ds = |z|^2 / eps + R P'(R); skipped where it is not above half of its
// kinetic part.
__device__ __forceinline__ void project_radially(double &zr, double &zv, double H0, double H1,
                                                 double RdP, double inv2eps)
{
    const double A = (zr * zr + zv * zv) * (2.0 * inv2eps);
    const double slope = A + RdP;
    if (slope > 0.5 * A) {
        const double s = 1.0 - (H1 - H0) / slope;
        zr *= s;
        zv *= s;
    }
}

// Waves per workgroup of the inference kernel.  With the Poisson field a
// workgroup holds a (N_r + 1)-entry histogram in LDS, which allows two
// workgroups per CU: eight waves each keep four waves on every SIMD.
constexpr int kWavesDuffing = 4, kWavesPoisson = 8;

// One learned step.  A workgroup of WAVES waves takes 64 WAVES particles per
// iteration, one per lane.  The network runs in two passes per wave, over the
// particles of lanes 0-31 and then of lanes 32-63; in each pass lanes c and
// c+32 share the particle of column c and split its k slots.  The update, the
// check and the projection then run once per particle, in its own lane.  All
// three layers run on MFMA (32x32x16, operand type T: FP16 or BF16, see
// InferOp) with FP32 accumulation:
//   layer 1  one MFMA per 32 hidden units; k slots 0-7 hold the features'
//            hi parts, the constant 1 (bias) and the features' lo parts
//            against the weights' hi parts, slots 8-15 the weights' lo parts
//            against the features' hi parts (FP16: ~22-bit, BF16: ~16-bit
//            products);
//   layer 2  W2 times the activations, accumulators started at the bias;
//   layer 3  W3 times the activations, lanes 0-31 receive the two outputs of
//            the pass's particle of their column (moved to lanes 32-63 in the
//            second pass).
// With FP16, W2 and W3 are not split: their 2^-12 rounding costs no
// measurable accuracy next to the activations' own, and splitting doubled
// those layers' MFMAs.
// The results of one layer are the next layer's B operand without any data
// movement: the k order of W2 and W3 is permuted at upload to the order in
// which the accumulator elements sit in the lanes.  Features are clamped to
// +-xmax (set from the weights so that no pre-activation can leave the FP16
// activation's range).  All weights stay in LDS and are read where used.  The
// update and the energy check run in FP64: H = |z|^2/(2 eps) + P(R) with
// P = R^4/4 (Duffing) or the frozen-field potential Psi^n (Poisson,
// VP = true).  The polar map acts around the base point: z_n itself (the
// free rotation) or, when c is given, the base push's result c_n (Duffing
// field).  With the amplitude-scaled output map the outputs are divided by
// a = |base point| first.  Particles that fail keep their state and go to the
// fallback queue.  With VP the sixth feature is E^n(R_n), and the particles
// that pass are deposited (CIC, fixed point) into an LDS histogram added to
// the mesh at the end.
// At most 128 VGPRs (four waves per SIMD): the split-BF16 forms would take
// 153 (Duffing) and 161 (Vlasov-Poisson), which leaves three waves per SIMD,
// and with eight-wave workgroups only one per CU.  The Vlasov-Poisson BF16
// form then spills nine registers and still runs 8 % faster.
template <bool VP, int WAVES, typename T>
__global__ __launch_bounds__(64 * WAVES, 4) void mlp_push_kernel(
    float *__restrict__ zR, float *__restrict__ zV, const float *__restrict__ cR,
    const float *__restrict__ cV, int64_t n, MlpInfer net, double2 rot0, double2 rot1,
    double inv2eps, double tol, unsigned *__restrict__ qcount, unsigned *__restrict__ queue,
    MeshView mv, PotView pv, const double *__restrict__ qb, unsigned long long *__restrict__ hist)
{
    const bool base = cR != nullptr;
    typedef InferOp<T> Op;
    typedef typename Op::vec vec;
    constexpr int kW = Op::kSplitW ? 2 : 1;   // weight parts of layers 2 and 3
    __shared__ uint4 sW2[kW * 8 * 64];
    __shared__ uint4 sW1[2 * 64];
    __shared__ float4 sb2[kH / 4];
    __shared__ uint4 sW3[kW * 4 * 64];
    __shared__ unsigned s_q[WAVES][kWaveQueue];
    extern __shared__ __align__(16) unsigned char vp_smem[];
    const int tid = threadIdx.x;
    for (int i = tid; i < kW * 8 * 64; i += blockDim.x) sW2[i] = net.w2f[i];
    if (tid < 2 * 64) sW1[tid] = net.w1f[tid];
    if (tid < kH / 4) sb2[tid] = net.b2[tid];
    for (int i = tid; i < kW * 4 * 64; i += blockDim.x) sW3[i] = net.w3f[i];
    if (VP) {
        mv.H = reinterpret_cast<unsigned long long *>(vp_smem);
        for (int i = tid; i <= pv.nr; i += blockDim.x) mv.H[i] = 0ull;
        mv.Qb = pv.Qb = *qb;
    }
    const int lane = tid & 63, wave = tid >> 6, g = lane >> 5;
    WaveQueue wq{s_q[wave], 0u};
    __syncthreads();

    constexpr int kGroup = 64 * WAVES;   // particles per workgroup iteration
    const int64_t nbg = (n + kGroup - 1) / kGroup;
    for (int64_t bg = blockIdx.x; bg < nbg; bg += gridDim.x) {
        // keep the LDS reads below inside the loop (no hoisting into registers)
        asm volatile("" ::: "memory");
        // lane l's own particle: the network passes below take those of lanes
        // 0-31 and then those of lanes 32-63; the update and the check run
        // once per particle, in its own lane
        const int64_t p = bg * kGroup + wave * 64 + lane;
        const bool valid = p < n;
        const double zr = valid ? (double)zR[p] : 0.0;
        const double zv = valid ? (double)zV[p] : 0.0;
        // base point of the polar map
        const double br = base && valid ? (double)cR[p] : zr;
        const double bv = base && valid ? (double)cV[p] : zv;
        const double R = fma(rot0.x, zr, rot0.y * zv);
        const double Vl = fma(-rot0.y, zr, rot0.x * zv);
        // features of the lane's particle, and of the particle in lane l ^ 32
        const float xf[3] = {(float)R, (float)Vl, VP ? (float)gather(mv, R) : 0.f};
        float xp[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) xp[i] = __shfl_xor(xf[i], 32, 64);
        float o0 = 0.f, o1 = 0.f;
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            // the weights stay in LDS across the passes too
            asm volatile("" ::: "memory");
            // pass h: particle 32 h + c in both lanes of column c = l mod 32;
            // the features, clamped, as hi + lo parts
            T xh[3], xl[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const float x = fminf(fmaxf(g == h ? xf[i] : xp[i], -net.xmax), net.xmax);
                xh[i] = (T)x;
                xl[i] = g == 0 ? (T)(x - (float)xh[i]) : (T)0.f;
            }
            const vec xb = {xh[0], xh[1], xh[2], (T)1.f, xl[0], xl[1], xl[2], (T)0.f};

            // layer 1: pre-activations / 64 of units 0-31 and 32-63
            const f32x16 zero = {};
            const f32x16 u0 = Op::mma(Op::load(sW1[lane]), xb, zero);
            const f32x16 u1 = Op::mma(Op::load(sW1[64 + lane]), xb, zero);
            // layer 2, accumulators started at b2 / 64
            f32x16 acc0, acc1;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float4 c0 = sb2[2 * j + g], c1 = sb2[8 + 2 * j + g];
                acc0[4 * j] = c0.x;
                acc0[4 * j + 1] = c0.y;
                acc0[4 * j + 2] = c0.z;
                acc0[4 * j + 3] = c0.w;
                acc1[4 * j] = c1.x;
                acc1[4 * j + 1] = c1.y;
                acc1[4 * j + 2] = c1.z;
                acc1[4 * j + 3] = c1.w;
            }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                vec b, lo;
                if constexpr (Op::kSplitA3)
                    b = Op::act_split(kk < 2 ? u0 : u1, 8 * (kk & 1), lo);
                else
                    b = Op::act(kk < 2 ? u0 : u1, 8 * (kk & 1));
#pragma unroll
                for (int w = 0; w < kW; ++w) {
                    acc0 = Op::mma(Op::load(sW2[(w * 8 + kk) * 64 + lane]), b, acc0);
                    acc1 = Op::mma(Op::load(sW2[(w * 8 + 4 + kk) * 64 + lane]), b, acc1);
                }
                if constexpr (Op::kSplitA3) {
                    acc0 = Op::mma(Op::load(sW2[kk * 64 + lane]), lo, acc0);
                    acc1 = Op::mma(Op::load(sW2[(4 + kk) * 64 + lane]), lo, acc1);
                }
            }
            // layer 3 (BF16: activations hi + lo as in layer 2)
            f32x16 acc3 = {};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                vec b, lo;
                if constexpr (Op::kSplitA3)
                    b = Op::act_split(kk < 2 ? acc0 : acc1, 8 * (kk & 1), lo);
                else
                    b = Op::act(kk < 2 ? acc0 : acc1, 8 * (kk & 1));
#pragma unroll
                for (int w = 0; w < kW; ++w)
                    acc3 = Op::mma(Op::load(sW3[(w * 4 + kk) * 64 + lane]), b, acc3);
                if constexpr (Op::kSplitA3) acc3 = Op::mma(Op::load(sW3[kk * 64 + lane]), lo, acc3);
            }
            // lanes 0-31 hold the outputs of pass h's particles; pass 1 moves
            // them to the particles' own lanes 32-63
            const float t0 = h ? __shfl_xor(acc3[0], 32, 64) : acc3[0];
            const float t1 = h ? __shfl_xor(acc3[1], 32, 64) : acc3[1];
            if (g == h) {
                o0 = t0;
                o1 = t1;
            }
        }
        float delta = fmaf(net.sig_d, o0 + net.b3_0, net.mu_d);
        const float kappa = fmaf(net.sig_k, o1 + net.b3_1, net.mu_k);
        double sc;
        if (net.scaled) {
            // outputs are (a delta, a kappa), divided by a = |z_b| in FP32
            // (both are FP32 values; 1/a to ~1 ulp costs nothing next to
            // them).  Nothing moves below a = 2^-50, where the scaled map is
            // void.
            const double a2 = fma(br, br, bv * bv);
            const float inv_a = a2 > 0x1p-100 ? rsqrtf((float)a2) : 0.f;
            delta *= inv_a;
            sc = 1.0 + (double)(kappa * inv_a);
        } else {
            sc = 1.0 + (double)kappa;
        }
        float sd, cd;
        sincosf(delta, &sd, &cd);
        double nr = sc * fma((double)cd, br, (double)sd * bv);
        double nv = sc * fma(-(double)sd, br, (double)cd * bv);
        const double R1 = fma(rot1.x, nr, rot1.y * nv);
        double P0, P1;
        if (VP) {
            P0 = potential(pv, R);
            P1 = potential(pv, R1);
        } else {
            P0 = 0.25 * (R * R) * (R * R);
            P1 = 0.25 * (R1 * R1) * (R1 * R1);
        }
        const double H0 = fma(zr * zr + zv * zv, inv2eps, P0);
        const double H1 = fma(nr * nr + nv * nv, inv2eps, P1);
        const bool ok = fabs(H1 - H0) <= tol * fabs(H0);
        if (net.project) {
            // one Newton step of the radial projection s y onto H = H0 from
            // s = 1: dH/ds = |y|^2 / eps + R P'(R), with R P'(R) = 4 P
            // (Duffing) or -R E^n(R) (Poisson); skipped where that slope is
            // below half its kinetic part (small orbits in the Poisson
            // field).  The correction is at most tol, so FP32 is ample for it.
            const double A = (nr * nr + nv * nv) * (2.0 * inv2eps);
            const double slope = VP ? fma(-R1, gather(mv, R1), A) : fma(4.0, P1, A);
            if (slope > 0.5 * A) {
                const float corr = (float)(H1 - H0) * __builtin_amdgcn_rcpf((float)slope);
                const double s = 1.0 - (double)corr;
                nr *= s;
                nv *= s;
            }
        }
        if (valid && ok) {
            const float fr = (float)nr, fv = (float)nv;
            zR[p] = fr;
            zV[p] = fv;
            if (VP) deposit(mv, fma(rot1.x, (double)fr, rot1.y * (double)fv));
        }
        wave_queue_push(wq, valid && !ok, (unsigned)p, qcount, queue, lane);
    }
    wave_queue_flush(wq, qcount, queue, lane);
    if (VP) {
        __syncthreads();
        const int nn = pv.nr + 1;
        const int start = (int)(((unsigned)blockIdx.x * 131u) % (unsigned)nn);
        for (int i0 = tid; i0 < nn; i0 += blockDim.x) {
            int i = i0 + start;
            if (i >= nn) i -= nn;
            const unsigned long long v = mv.H[i];
            if (v) atomicAdd(&hist[i], v);
        }
    }
}

// Fallback kernels keep the substep coefficients in LDS up to this many
// substeps (64 KB); beyond it they read them from global memory.
constexpr int kFallbackLdsK = 2048;
// The Duffing fallback holds nothing else in LDS, so its table may take up
// to 128 KB: the fallback of the base-push network runs K_fb = 3200 substeps.
constexpr int kFallbackLdsKDuffing = 4096;

// LDS of the Poisson fallback: field table and histogram, as in the mesh push
// kernel, then the coefficient table at a 32-byte boundary.
__host__ __device__ constexpr size_t fallback_table_offset(int nr)
{
    return ((size_t)nr * sizeof(float2) + (size_t)(nr + 1) * sizeof(unsigned long long) + 31) &
           ~(size_t)31;
}

// K substeps of the plain push of one particle.  A fallback kernel holds few
// particles, so its loop is bound by latency: the substep coefficients are
// read eight substeps at a time (one wait per eight table reads instead of
// one per substep).  Same arithmetic in the same order as the plain push
// kernels, so a fallback particle gets exactly the plain push.
template <typename Field>
__device__ __forceinline__ void push_staged(const double4 *__restrict__ t, int K, Field field,
                                            double &zr, double &zv)
{
    double ar = 0.0, av = 0.0;
    const auto substep = [&](const double4 &q) {
        const double Rm = fma(q.x, zr + ar, q.y * (zv + av));
        const double E = field(Rm);
        ar = fma(-q.z, E, ar);
        av = fma(q.w, E, av);
    };
    int k = 0;
    for (; k + 8 <= K; k += 8) {
        double4 q[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) q[j] = t[k + j];
#pragma unroll
        for (int j = 0; j < 8; ++j) substep(q[j]);
    }
    for (; k < K; ++k) substep(t[k]);
    zr += ar;
    zv += av;
}

// Fallback threads take the queue entries i = b + G (t + T j), j = 0, 1, ...
// (b the workgroup, t the thread, T threads per workgroup): entry i goes to
// workgroup i mod G, so that a short queue still spreads over every CU (each
// wave of a fallback runs K dependent substeps, and waves that share a SIMD
// wait on each other).  G is at least min_groups (one per CU) and otherwise
// the workgroups the queue fills, up to the grid: each workgroup that takes
// entries first stages the coefficient table, so a short queue wakes no more
// of them than it needs.
__device__ __forceinline__ unsigned fallback_groups(unsigned count, unsigned min_groups)
{
    const uint64_t need = ((uint64_t)count + blockDim.x - 1) / blockDim.x;
    const uint64_t g = need > min_groups ? need : min_groups;
    return g < gridDim.x ? (unsigned)g : gridDim.x;
}

// Copies the K substep coefficients into LDS (K within the kernel's limit).
__device__ __forceinline__ double4 *stage_table(unsigned char *smem, const double4 *sub, int K)
{
    double4 *t = reinterpret_cast<double4 *>(smem);
    for (int i = threadIdx.x; i < K; i += blockDim.x) t[i] = sub[i];
    return t;
}

// Plain push (K substeps, FP64) of the queued particles, Duffing field.
// Workgroups past the queue's end return at once; the others stage the
// coefficient table in LDS when it fits (K <= kFallbackLdsKDuffing).
__global__ __launch_bounds__(256) void fallback_duffing_kernel(
    float *__restrict__ zR, float *__restrict__ zV, const unsigned *__restrict__ queue,
    const unsigned *__restrict__ qcount, const double4 *__restrict__ sub, int K,
    FallbackProjection proj, unsigned long long *__restrict__ total, unsigned min_groups)
{
    extern __shared__ __align__(16) unsigned char fbd_smem[];
    const unsigned count = *qcount;
    if (blockIdx.x == 0 && threadIdx.x == 0) *total += count;
    const unsigned G = fallback_groups(count, min_groups);
    if ((unsigned)blockIdx.x >= G || (unsigned)blockIdx.x >= count) return;   // uniform
    const auto duffing = [](double R) { return -(R * R) * R; };
    const auto run = [&](const double4 *t) {
        for (uint64_t i = blockIdx.x + (uint64_t)threadIdx.x * G; i < count;
             i += (uint64_t)blockDim.x * G) {
            const unsigned p = queue[i];
            double zr = zR[p], zv = zV[p];
            double H0 = 0.0;
            if (proj.on) {
                const double R0 = fma(proj.rot0.x, zr, proj.rot0.y * zv);
                H0 = fma(zr * zr + zv * zv, proj.inv2eps, 0.25 * (R0 * R0) * (R0 * R0));
            }
            push_staged(t, K, duffing, zr, zv);
            if (proj.on) {
                const double R1 = fma(proj.rot1.x, zr, proj.rot1.y * zv);
                const double P1 = 0.25 * (R1 * R1) * (R1 * R1);
                project_radially(zr, zv, H0, fma(zr * zr + zv * zv, proj.inv2eps, P1), 4.0 * P1,
                                 proj.inv2eps);
            }
            zR[p] = (float)zr;
            zV[p] = (float)zv;
        }
    };
    // two loops, so that each one's table reads use their own address space
    if (K <= kFallbackLdsKDuffing) {
        const double4 *t = stage_table(fbd_smem, sub, K);
        __syncthreads();
        run(t);
    } else {
        run(sub);
    }
}

// Plain push (K substeps, FP64, field table and, when it fits, the substep
// coefficients in LDS) of the queued particles in the frozen Poisson field,
// then their CIC deposit at the end-of-step phase.
__global__ __launch_bounds__(kPushBlock) void fallback_poisson_kernel(
    float *__restrict__ zR, float *__restrict__ zV, const unsigned *__restrict__ queue,
    const unsigned *__restrict__ qcount, const double4 *__restrict__ sub, int K, double2 er,
    MeshView mv, PotView pv, FallbackProjection proj, const float2 *__restrict__ etab,
    const double *__restrict__ fscal, int nr, unsigned long long *__restrict__ hist,
    unsigned long long *__restrict__ total, unsigned min_groups)
{
    extern __shared__ __align__(16) unsigned char fb_smem[];
    const unsigned count = *qcount;
    if (blockIdx.x == 0 && threadIdx.x == 0) *total += count;
    // uniform over the workgroup: an empty workgroup has nothing to deposit
    const unsigned G = fallback_groups(count, min_groups);
    if ((unsigned)blockIdx.x >= G || (unsigned)blockIdx.x >= count) return;
    const int tid = threadIdx.x;
    mv.Et = reinterpret_cast<float2 *>(fb_smem);
    mv.H = reinterpret_cast<unsigned long long *>(fb_smem + (size_t)nr * sizeof(float2));
    float2 *Et = reinterpret_cast<float2 *>(fb_smem);
    for (int i = tid; i < nr; i += blockDim.x) Et[i] = etab[i];
    for (int i = tid; i <= nr; i += blockDim.x) mv.H[i] = 0ull;
    mv.Qb = pv.Qb = fscal[kQb];
    const bool staged = K <= kFallbackLdsK;
    const double4 *t = staged ? stage_table(fb_smem + fallback_table_offset(nr), sub, K) : nullptr;
    // particles with |z|^2 < lim2 take the gather without range tests
    const double lim2 = on_mesh_limit2(mv, sub, K, fscal[kEmax]);
    __syncthreads();
    const auto field = [&mv](double R) { return gather(mv, R); };
    const auto field_on = [&mv](double R) { return gather_on(mv, R); };
    const auto run = [&](const double4 *tab) {
        for (uint64_t i = blockIdx.x + (uint64_t)threadIdx.x * G; i < count;
             i += (uint64_t)blockDim.x * G) {
            const unsigned p = queue[i];
            double zr = zR[p], zv = zV[p];
            double H0 = 0.0;
            if (proj.on) {
                const double R0 = fma(proj.rot0.x, zr, proj.rot0.y * zv);
                H0 = fma(zr * zr + zv * zv, proj.inv2eps, potential(pv, R0));
            }
            if (fma(zr, zr, zv * zv) < lim2)
                push_staged(tab, K, field_on, zr, zv);
            else
                push_staged(tab, K, field, zr, zv);
            if (proj.on) {
                const double R1 = fma(er.x, zr, er.y * zv);
                project_radially(zr, zv, H0,
                                 fma(zr * zr + zv * zv, proj.inv2eps, potential(pv, R1)),
                                 -R1 * gather(mv, R1), proj.inv2eps);
            }
            const float fr = (float)zr, fv = (float)zv;
            zR[p] = fr;
            zV[p] = fv;
            deposit(mv, fma(er.x, (double)fr, er.y * (double)fv));
        }
    };
    // two loops, so that each one's table reads use their own address space
    if (staged)
        run(t);
    else
        run(sub);
    __syncthreads();
    const int nn = nr + 1;
    const int start = (int)(((unsigned)blockIdx.x * 131u) % (unsigned)nn);
    for (int i0 = tid; i0 < nn; i0 += blockDim.x) {
        int i = i0 + start;
        if (i >= nn) i -= nn;
        const unsigned long long v = mv.H[i];
        if (v) atomicAdd(&hist[i], v);
    }
}

static MeshView mesh_view(const MeshArgs &ma)
{
    MeshView m;
    m.Et = ma.etab;
    m.H = nullptr;
    m.inv_hr = 1.0 / ma.hr;
    m.half = 0.5 * (double)ma.nr;
    m.c = ma.nr >> 1;
    m.Qb = 0.0;
    return m;
}

hipError_t launch_mlp_push_duffing(hipStream_t st, float *zR, float *zV, const float *cR,
                                   const float *cV, int64_t n, const MlpInfer &net, double2 rot0,
                                   double2 rot1, double eps, double tol, unsigned *qcount,
                                   unsigned *queue, int n_cu)
{
    if (n <= 0) return hipSuccess;
    int64_t grid = (n + 64 * kWavesDuffing - 1) / (64 * kWavesDuffing);
    if (grid > (int64_t)n_cu * 8) grid = (int64_t)n_cu * 8;
    const dim3 g((unsigned)grid), b(64 * kWavesDuffing);
    if (net.fp16)
        return dispatch(mlp_push_kernel<false, kWavesDuffing, _Float16>, g, b, 0, st, zR, zV, cR,
                        cV, n, net, rot0, rot1, 0.5 / eps, tol, qcount, queue, MeshView{},
                        PotView{}, (const double *)nullptr, (unsigned long long *)nullptr);
    return dispatch(mlp_push_kernel<false, kWavesDuffing, __bf16>, g, b, 0, st, zR, zV, cR, cV, n,
                    net, rot0, rot1, 0.5 / eps, tol, qcount, queue, MeshView{}, PotView{},
                    (const double *)nullptr, (unsigned long long *)nullptr);
}

static size_t mlp_vp_lds_bytes(int nr) { return (size_t)(nr + 1) * sizeof(unsigned long long); }

// The FP64 node field and potential of the mesh (Qb is read on the device).
static PotView pot_view(const MeshArgs &ma, double rmax)
{
    PotView pv;
    pv.E = ma.E64;
    pv.Psi = ma.Psi64;
    pv.hr = ma.hr;
    pv.inv_hr = 1.0 / ma.hr;
    pv.half = 0.5 * (double)ma.nr;
    pv.rmax = rmax;
    pv.Qb = 0.0;
    pv.c = ma.nr >> 1;
    pv.nr = ma.nr;
    return pv;
}

hipError_t launch_mlp_push_poisson(hipStream_t st, float *zR, float *zV, int64_t n,
                                   const MlpInfer &net, double2 rot0, double2 rot1, double eps,
                                   double tol, unsigned *qcount, unsigned *queue,
                                   const MeshArgs &ma, double rmax, int n_cu)
{
    if (n <= 0) return hipSuccess;
    int64_t grid = (n + 64 * kWavesPoisson - 1) / (64 * kWavesPoisson);
    if (grid > (int64_t)n_cu * 2) grid = (int64_t)n_cu * 2;
    const PotView pv = pot_view(ma, rmax);
    const dim3 g((unsigned)grid), b(64 * kWavesPoisson);
    const size_t lds = mlp_vp_lds_bytes(ma.nr);
    if (net.fp16)
        return dispatch(mlp_push_kernel<true, kWavesPoisson, _Float16>, g, b, lds, st, zR, zV,
                        (const float *)nullptr, (const float *)nullptr, n, net, rot0, rot1,
                        0.5 / eps, tol, qcount, queue, mesh_view(ma), pv,
                        (const double *)(ma.fscal + kQb), ma.hist);
    return dispatch(mlp_push_kernel<true, kWavesPoisson, __bf16>, g, b, lds, st, zR, zV,
                    (const float *)nullptr, (const float *)nullptr, n, net, rot0, rot1,
                    0.5 / eps, tol, qcount, queue, mesh_view(ma), pv,
                    (const double *)(ma.fscal + kQb), ma.hist);
}

hipError_t launch_fallback_duffing(hipStream_t st, float *zR, float *zV, const unsigned *queue,
                                   const unsigned *qcount, const double4 *sub, int K,
                                   const FallbackProjection &proj, unsigned long long *total,
                                   int n_cu)
{
    const size_t lds = K <= kFallbackLdsKDuffing ? (size_t)K * sizeof(double4) : 0;
    return dispatch(fallback_duffing_kernel, dim3((unsigned)n_cu * 8), dim3(256), lds, st, zR, zV,
                    queue, qcount, sub, K, proj, total, (unsigned)n_cu);
}

hipError_t launch_fallback_poisson(hipStream_t st, float *zR, float *zV, const unsigned *queue,
                                   const unsigned *qcount, const double4 *sub, int K, double2 er,
                                   const MeshArgs &ma, double rmax, const FallbackProjection &proj,
                                   unsigned long long *total, int n_cu)
{
    const size_t lds = K <= kFallbackLdsK
                           ? fallback_table_offset(ma.nr) + (size_t)K * sizeof(double4)
                           : push_lds_bytes_for(ma.nr);
    return dispatch(fallback_poisson_kernel, dim3((unsigned)n_cu), dim3(kPushBlock), lds, st, zR, zV,
                    queue, qcount, sub, K, er, mesh_view(ma), pot_view(ma, rmax), proj,
                    (const float2 *)ma.etab, (const double *)ma.fscal, ma.nr, ma.hist, total,
                    (unsigned)n_cu);
}

hipError_t setup_learned_lds(int nr)
{
    hipError_t e = raise_dynamic_lds(
        reinterpret_cast<const void *>(&mlp_push_kernel<true, kWavesPoisson, _Float16>),
        (int)mlp_vp_lds_bytes(nr));
    if (e != hipSuccess) return e;
    e = raise_dynamic_lds(
        reinterpret_cast<const void *>(&mlp_push_kernel<true, kWavesPoisson, __bf16>),
        (int)mlp_vp_lds_bytes(nr));
    if (e != hipSuccess) return e;
    e = raise_dynamic_lds(reinterpret_cast<const void *>(&fallback_duffing_kernel),
                          (int)(kFallbackLdsKDuffing * sizeof(double4)));
    if (e != hipSuccess) return e;
    return raise_dynamic_lds(reinterpret_cast<const void *>(&fallback_poisson_kernel),
                             (int)(fallback_table_offset(nr) + kFallbackLdsK * sizeof(double4)));
}

}  // namespace etd
