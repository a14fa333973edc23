// HIP kernels of the plain exponential-integrator PIC step (gfx950).
//
// State: SoA FP32 arrays zR, zV holding the particle state in the frame that
// rotates with the free flow, z = r(-t/eps) y, r the rotation of eq. 3.3 with
// T = 2 pi.  In that frame the stiff linear part of eq. 3.1 drops out and
// eq. 3.6 becomes dz/dt = r(-t/eps) (0, E(R, t)), R = [r(t/eps) z]_R, so the
// exact rotation is never applied to the stored state; the fast phase t/eps is
// carried in FP64 and only enters through per-substep (cos, sin) tables.
//
// Push (one macro step dt = K h, field frozen at t_n): midpoint rule for the
// Duhamel integral of eq. 3.6 on each substep,
//     R_mid = cos(phi_k) zR + sin(phi_k) zV,  E = E(R_mid),
//     zR -= h sin(phi_k) E,  zV += h cos(phi_k) E,
// phi_k the phase at the substep midpoint.  With E = 0 the state is unchanged,
// which is the exact free rotation of period 2 pi eps.
//
// Precision: the state is stored in FP32 (16 bytes of HBM traffic per
// particle-step); in registers every push does its arithmetic in FP64, which
// on CDNA runs at the rate of non-packed FP32 FMAs.  The FP64 cell coordinate
// keeps the CIC weights exact to the stored positions even next to the steep
// centre cell of the field, and the substep increments are accumulated
// without FP32 cancellation.  Only the tabulated field is FP32.
//
// Mesh: N_r cells on [-r_max, r_max], nodes x_k = (k - N_r/2) h_r.  Cell
// coordinates are taken relative to the centre node, x = R / h_r.  The CIC
// deposit accumulates the two node weights (1 - th, th) of every particle as
// integers in units of 2^-32 of a particle weight, in LDS per workgroup and
// then into one global u64 histogram; integer sums make the charge, and
// therefore the whole step, independent of the order of accumulation.  The
// Poisson solve (section 2.3: trapezoidal rule on the cells) runs on those
// integers: the trapezoid prefix sum of the node charges is an exact integer
// scan.

#include "pic_device.h"

typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace etd {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// ------------------------------------------------------------ phase tables

// Coefficients of steps j0 .. j0 + S - 1 counted from the phase phi0: step j
// starts at fmod(phi0 + j dphi, 2 pi); entry (j - j0) K + k holds substep k.
__global__ void phase_table_kernel(double4 *__restrict__ sub, double2 *__restrict__ endrot,
                                   double phi0, double dphi, double theta, double h, int K,
                                   int S, int64_t j0)
{
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)S * K;
    if (idx < total) {
        const int64_t j = idx / K;
        const int64_t k = idx - j * K;
        const double pj = fmod(phi0 + (double)(j0 + j) * dphi, kTwoPi);
        const double ph = pj + ((double)k + 0.5) * theta;
        double s, c;
        sincos(ph, &s, &c);
        sub[idx] = make_double4(c, s, h * s, h * c);
    }
    if (idx < S) {
        const double p1 = fmod(phi0 + (double)(j0 + idx + 1) * dphi, kTwoPi);
        double s, c;
        sincos(p1, &s, &c);
        endrot[idx] = make_double2(c, s);
    }
}

hipError_t launch_phase_table(hipStream_t st, StepTables tab, double phi0, double dphi,
                              double theta, double h, int K, int S, int64_t j0)
{
    const int64_t total = (int64_t)S * K > S ? (int64_t)S * K : S;
    const int block = 256;
    const int64_t grid = (total + block - 1) / block;
    phase_table_kernel<<<dim3((unsigned)grid), dim3(block), 0, st>>>(tab.sub, tab.endrot, phi0,
                                                                   dphi, theta, h, K, S, j0);
    return hipGetLastError();
}

// ------------------------------------------------------------ frame changes

// z = r(-phi) y : zR = c R - s V, zV = s R + c V   (FP64, rounded once)
__global__ void twist_in_kernel(const double *__restrict__ R, const double *__restrict__ V,
                                float *__restrict__ zR, float *__restrict__ zV, int64_t n,
                                double c, double s)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        const double r = R[i], v = V[i];
        zR[i] = (float)(c * r - s * v);
        zV[i] = (float)(s * r + c * v);
    }
}

// y = r(phi) z : R = c zR + s zV, V = -s zR + c zV   (FP64)
__global__ void twist_out_kernel(const float *__restrict__ zR, const float *__restrict__ zV,
                                 double *__restrict__ R, double *__restrict__ V, int64_t n,
                                 double c, double s)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        const double r = zR[i], v = zV[i];
        R[i] = c * r + s * v;
        V[i] = -s * r + c * v;
    }
}

hipError_t launch_twist_in(hipStream_t st, const double *R, const double *V, float *zR,
                           float *zV, int64_t n, double c, double s)
{
    if (n <= 0) return hipSuccess;
    const int block = 256;
    twist_in_kernel<<<dim3((unsigned)((n + block - 1) / block)), dim3(block), 0, st>>>(
        R, V, zR, zV, n, c, s);
    return hipGetLastError();
}

hipError_t launch_twist_out(hipStream_t st, const float *zR, const float *zV, double *R,
                            double *V, int64_t n, double c, double s)
{
    if (n <= 0) return hipSuccess;
    const int block = 256;
    twist_out_kernel<<<dim3((unsigned)((n + block - 1) / block)), dim3(block), 0, st>>>(
        zR, zV, R, V, n, c, s);
    return hipGetLastError();
}

// ------------------------------------------------------------ Duffing push

// E = -R^3 needs no mesh, so particles are independent: each lane keeps its
// state in FP64 registers for all S steps of the launch and rounds it to FP32
// once, at the store.
__global__ __launch_bounds__(256) void push_duffing_kernel(float *__restrict__ zR,
                                                           float *__restrict__ zV, int64_t n,
                                                           const double4 *__restrict__ sub,
                                                           int K, int S)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double zr = zR[i], zv = zV[i];
    const double4 *t = sub;
    for (int j = 0; j < S; ++j) {
        double ar = 0.0, av = 0.0;
        for (int k = 0; k < K; ++k) {
            const double4 q = t[k];
            const double Rm = fma(q.x, zr + ar, q.y * (zv + av));
            const double E = -(Rm * Rm) * Rm;
            ar = fma(-q.z, E, ar);
            av = fma(q.w, E, av);
        }
        t += K;
        zr += ar;
        zv += av;
    }
    zR[i] = (float)zr;
    zV[i] = (float)zv;
}

hipError_t launch_push_duffing(hipStream_t st, float *zR, float *zV, int64_t n,
                               const double4 *sub, int K, int S)
{
    if (n <= 0 || S <= 0) return hipSuccess;
    const int block = 256;
    return dispatch(push_duffing_kernel, dim3((unsigned)((n + block - 1) / block)), dim3(block), 0,
                    st, zR, zV, n, sub, K, S);
}

// ------------------------------------------------------------ mesh solve

// One workgroup.  From the fixed-point node charges S_k (units of 2^-32 w):
//   rho_k = w 2^-32 S_k / h_r                                   (CIC density)
//   I_k   = sum_{i=1..k} (S_{i-1} + S_i)        exact integer trapezoid scan,
//           so P_k = int_{x_0}^{x_k} rho = w 2^-33 I_k
//   Q_j   = (P_{c+j} - P_{c-j}) / 2 = w 2^-34 (I_{c+j} - I_{c-j})
//   E_k   = Q_{|k-c|} / x_k  (k != c),  E_c = 0,  Qb = w 2^-34 I_nr
// and the FP32 gather table (E_m, E_{m+1} - E_m), with the bound
// emax = max |E_k| (1 + 2^-20) on the gathered field (a gather lies between
// the table's node values, which are within 3 2^-24 max |E_k| of the FP64
// ones).  Clears hist for the next
// accumulation.  Node arrays live in the caller's LDS (2 (nr+1) u64): S and
// I as u64, then E as FP64 in the storage of S.  Elementwise passes run
// node-contiguous across threads; the scan runs over contiguous per-thread
// chunks.  Leaves E in LDS (first nr+1 doubles) for solve_potential_block.
__device__ void solve_field_block(unsigned char *smem, unsigned long long *__restrict__ hist,
                                  int nr, double w, double hr, float2 *__restrict__ etab,
                                  double *__restrict__ rho64, double *__restrict__ E64,
                                  double *__restrict__ fscal)
{
    const int nn = nr + 1;
    unsigned long long *S = reinterpret_cast<unsigned long long *>(smem);
    double *Ed = reinterpret_cast<double *>(smem);
    unsigned long long *I = S + nn;
    __shared__ unsigned long long wu[kSolveBlock / 64];
    __shared__ unsigned long long emax_bits;   // max |E_k| as FP64 bits (ordered for x >= 0)
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid == 0) emax_bits = 0ull;   // visible after the scan's barriers
    const int c = nr >> 1;
    const double rho_scale = w * kFixScale / hr;

    // four loads in flight per thread (clamped to the last node; a clamped
    // duplicate is read, never stored), then their stores
#pragma unroll 1
    for (int kb = tid; kb < nn; kb += 4 * nt) {
        unsigned long long v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = hist[min(kb + j * nt, nn - 1)];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = kb + j * nt;
            if (k < nn) {
                S[k] = v[j];
                rho64[k] = (double)v[j] * rho_scale;
                hist[k] = 0ull;
            }
        }
    }
    __syncthreads();

    const int chunk = (nn + nt - 1) / nt;
    const int k0 = min(tid * chunk, nn), k1 = min(k0 + chunk, nn);
    unsigned long long loc = 0ull, charge = 0ull;
#pragma unroll 1
    for (int k = k0; k < k1; ++k) {
        charge += S[k];
        if (k > 0) loc += S[k - 1] + S[k];
    }
    unsigned long long run = block_exclusive_scan<unsigned long long>(loc, wu);
#pragma unroll 1
    for (int k = k0; k < k1; ++k) {
        if (k > 0) run += S[k - 1] + S[k];
        I[k] = run;
    }
    charge = block_sum<unsigned long long>(charge, wu);   // syncs: I is complete

    const double q_scale = w * kFixScale * 0.25;
    double emax = 0.0;
#pragma unroll 1
    for (int k = tid; k < nn; k += nt) {
        double E = 0.0;
        if (k != c) {
            const int j = k > c ? k - c : c - k;
            const double Q = (double)(I[c + j] - I[c - j]) * q_scale;
            E = Q / ((double)(k - c) * hr);
        }
        Ed[k] = E;
        E64[k] = E;
        emax = fmax(emax, fabs(E));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) emax = fmax(emax, __shfl_xor(emax, off, 64));
    if ((tid & 63) == 0) atomicMax(&emax_bits, (unsigned long long)__double_as_longlong(emax));
    if (tid == 0) {
        fscal[kQb] = (double)I[nr] * q_scale;
        fscal[kMeshCharge] = (double)charge * w * kFixScale;
    }
    __syncthreads();
    if (tid == 0) fscal[kEmax] = __longlong_as_double((long long)emax_bits) * (1.0 + 0x1p-20);

#pragma unroll 1
    for (int k = tid; k < nr; k += nt) {
        const double e0 = Ed[k], e1 = Ed[k + 1];
        etab[k] = make_float2((float)e0, (float)(e1 - e0));
    }
}

// From the node field E in LDS (first nr+1 doubles of smem; the next nr+1
// are scratch), with every thread past a barrier since E was written:
//   Psi_k = -int_0^{x_k} E  (trapezoid of the node values)
//   field energy int_0^{r_max} x E^2 dx (trapezoid)
// in a fixed summation order, so that the potential kernel and the full solve
// give the same bits.
__device__ void solve_potential_block(unsigned char *smem, int nr, double hr,
                                      double *__restrict__ Psi64, double *__restrict__ fscal)
{
    const int nn = nr + 1;
    const double *Ed = reinterpret_cast<const double *>(smem);
    double *Fd = reinterpret_cast<double *>(smem) + nn;
    __shared__ double wd[kSolveBlock / 64];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int c = nr >> 1;
    const int chunk = (nn + nt - 1) / nt;
    const int k0 = min(tid * chunk, nn), k1 = min(k0 + chunk, nn);

    double fe = 0.0;
#pragma unroll 1
    for (int k = tid; k < nr; k += nt) {
        if (k >= c) {
            const double e0 = Ed[k], e1 = Ed[k + 1];
            const double x0 = (double)(k - c) * hr, x1 = (double)(k + 1 - c) * hr;
            fe += hr * (x0 * e0 * e0 + x1 * e1 * e1) * 0.5;
        }
    }
    // potential: F_k = sum_{i=1..k} h_r (E_{i-1} + E_i) / 2,  Psi_k = -(F_k - F_c)
    double locd = 0.0;
#pragma unroll 1
    for (int k = k0; k < k1; ++k)
        if (k > 0) locd += hr * (Ed[k - 1] + Ed[k]) * 0.5;
    double runf = block_exclusive_scan<double>(locd, wd);
#pragma unroll 1
    for (int k = k0; k < k1; ++k) {
        if (k > 0) runf += hr * (Ed[k - 1] + Ed[k]) * 0.5;
        Fd[k] = runf;
    }
    fe = block_sum<double>(fe, wd);   // syncs: Fd is complete
    const double Fc = Fd[c];
#pragma unroll 1
    for (int k = tid; k < nn; k += nt) Psi64[k] = -(Fd[k] - Fc);
    if (tid == 0) fscal[kFieldEnergy] = fe;
}

// The field (and with POT its potential and energy) of the accumulated charge.
template <bool POT>
__global__ __launch_bounds__(kSolveBlock) void mesh_solve_kernel(
    unsigned long long *__restrict__ hist, int nr, double w, double hr, float2 *__restrict__ etab,
    double *__restrict__ rho64, double *__restrict__ E64, double *__restrict__ Psi64,
    double *__restrict__ fscal)
{
    extern __shared__ __align__(16) unsigned char smem[];
    solve_field_block(smem, hist, nr, w, hr, etab, rho64, E64, fscal);
    if (POT) solve_potential_block(smem, nr, hr, Psi64, fscal);
}

// The potential and field energy of the field in E64.
__global__ __launch_bounds__(kSolveBlock) void potential_kernel(const double *__restrict__ E64,
                                                                int nr, double hr,
                                                                double *__restrict__ Psi64,
                                                                double *__restrict__ fscal)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double *Ed = reinterpret_cast<double *>(smem);
    const int nt = blockDim.x;
    // four loads in flight per thread (clamped to the last node)
#pragma unroll 1
    for (int kb = threadIdx.x; kb <= nr; kb += 4 * nt) {
        double v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = E64[min(kb + j * nt, nr)];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (kb + j * nt <= nr) Ed[kb + j * nt] = v[j];
    }
    __syncthreads();
    solve_potential_block(smem, nr, hr, Psi64, fscal);
}

static size_t mesh_lds_bytes(int nr) { return (size_t)2 * (nr + 1) * sizeof(unsigned long long); }

hipError_t launch_mesh_solve(hipStream_t st, const MeshArgs &a, bool potential)
{
    if (potential)
        return dispatch(mesh_solve_kernel<true>, dim3(1), dim3(kSolveBlock), mesh_lds_bytes(a.nr),
                        st, a.hist, a.nr, a.w, a.hr, a.etab, a.rho64, a.E64, a.Psi64, a.fscal);
    return dispatch(mesh_solve_kernel<false>, dim3(1), dim3(kSolveBlock), mesh_lds_bytes(a.nr), st,
                    a.hist, a.nr, a.w, a.hr, a.etab, a.rho64, a.E64, a.Psi64, a.fscal);
}

hipError_t launch_potential(hipStream_t st, const MeshArgs &a)
{
    return dispatch(potential_kernel, dim3(1), dim3(kSolveBlock), mesh_lds_bytes(a.nr), st,
                    (const double *)a.E64, a.nr, a.hr, a.Psi64, a.fscal);
}

// ------------------------------------------------------------ Poisson push + deposit

// One macro step of a tile of particles: load FP32 state, K-substep push in
// the frozen field (PUSH), store, and deposit the new positions -- rounded
// to the stored FP32 state, so that a later deposit of the same state gives
// the same charge bit for bit.
template <bool PUSH, int U>
__global__ __launch_bounds__(kPushBlock) void push_poisson_kernel(
    float *__restrict__ zR, float *__restrict__ zV, int64_t n, const double4 *__restrict__ sub,
    const double2 *__restrict__ endrot_tab, double2 endrot_val, int K, double inv_hr, MeshArgs ma)
{
    const int nr = ma.nr;
    const float2 *__restrict__ etab = ma.etab;
    unsigned long long *__restrict__ hist = ma.hist;
    extern __shared__ __align__(16) unsigned char smem[];
    float2 *Et = reinterpret_cast<float2 *>(smem);
    unsigned long long *H = reinterpret_cast<unsigned long long *>(smem + (size_t)nr * sizeof(float2));
    const int tid = threadIdx.x;
    if (PUSH)
        for (int i = tid; i < nr; i += blockDim.x) Et[i] = etab[i];
    for (int i = tid; i <= nr; i += blockDim.x) H[i] = 0ull;
    MeshView m;
    m.Et = Et;
    m.H = H;
    m.inv_hr = inv_hr;
    m.half = 0.5 * (double)nr;
    m.c = nr >> 1;
    m.Qb = PUSH ? ma.fscal[kQb] : 0.0;
    const double2 er = endrot_tab ? endrot_tab[0] : endrot_val;
    // particles with |z|^2 < lim2 take the gather without range tests.  Only
    // the two-group form, which the launcher takes for long state streams:
    // its table reads in flight together need many resident waves to hide
    // their latency, and with the one-group form's short grids (under two
    // workgroups per CU) the branch-free loop measured 20-30 % slower.
    constexpr bool kFast = PUSH && U == 2;
    const double lim2 = kFast ? on_mesh_limit2(m, sub, K, ma.fscal[kEmax]) : -1.0;
    __syncthreads();

    // Each thread takes U float4 groups (4 U particles) per iteration, with
    // all their loads in flight before any arithmetic.  The state is streamed
    // once per step, so loads and stores are nontemporal: they do not displace
    // the field table and histogram lines that the caches hold.
    const int64_t n4 = n >> 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * U;
    f32x4 *zR4 = reinterpret_cast<f32x4 *>(zR);
    f32x4 *zV4 = reinterpret_cast<f32x4 *>(zV);
    for (int64_t g0 = blockIdx.x * (int64_t)blockDim.x * U + tid; g0 < n4; g0 += stride) {
        f32x4 r4[U], v4[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = g0 + (int64_t)u * blockDim.x;
            if (i < n4) {
                r4[u] = __builtin_nontemporal_load(&zR4[i]);
                v4[u] = __builtin_nontemporal_load(&zV4[i]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = g0 + (int64_t)u * blockDim.x;
            if (i < n4) {
                f32x4 fr = r4[u], fv = v4[u];
                if (PUSH) {
                    double zr[4], zv[4];
                    bool on = true;
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        zr[p] = fr[p];
                        zv[p] = fv[p];
                        on = on && fma(zr[p], zr[p], zv[p] * zv[p]) < lim2;
                    }
                    if (kFast && on)
                        push_group<4, true>(m, sub, K, zr, zv);
                    else
                        push_group<4>(m, sub, K, zr, zv);
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        fr[p] = (float)zr[p];
                        fv[p] = (float)zv[p];
                    }
                    __builtin_nontemporal_store(fr, &zR4[i]);
                    __builtin_nontemporal_store(fv, &zV4[i]);
                }
#pragma unroll
                for (int p = 0; p < 4; ++p)
                    deposit(m, fma(er.x, (double)fr[p], er.y * (double)fv[p]));
            }
        }
    }
    // ragged tail: the last n % 4 particles
    const int64_t gt = blockIdx.x * (int64_t)blockDim.x + tid;
    const int64_t tail = n - (n4 << 2);
    if (gt < tail) {
        const int64_t i = (n4 << 2) + gt;
        float fr = zR[i], fv = zV[i];
        if (PUSH) {
            double zr[1] = {fr};
            double zv[1] = {fv};
            push_group<1>(m, sub, K, zr, zv);
            fr = (float)zr[0];
            fv = (float)zv[0];
            zR[i] = fr;
            zV[i] = fv;
        }
        deposit(m, fma(er.x, (double)fr, er.y * (double)fv));
    }
    __syncthreads();
    // flush: each workgroup starts at its own node offset so that concurrent
    // workgroups add to different addresses
    const int nn = nr + 1;
    const int start = (int)(((unsigned)blockIdx.x * 131u) % (unsigned)nn);
    for (int i0 = tid; i0 < nn; i0 += blockDim.x) {
        int i = i0 + start;
        if (i >= nn) i -= nn;
        const unsigned long long v = H[i];
        if (v) atomicAdd(&hist[i], v);
    }
}

// field table + histogram
static size_t push_lds_bytes(int nr)
{
    return (size_t)nr * sizeof(float2) + (size_t)(nr + 1) * sizeof(unsigned long long);
}

hipError_t launch_push_poisson(hipStream_t st, bool push, float *zR, float *zV, int64_t n,
                               const double4 *sub, const double2 *endrot_tab, double2 endrot_val,
                               int K, const MeshArgs &ma, int grid_cap)
{
    if (n <= 0) return hipSuccess;
    const size_t lds = push_lds_bytes(ma.nr);
    const int64_t n4 = n >> 2;
    // Two float4 groups per thread keep more loads in flight where the state
    // stream is long; a short one would leave CUs without a workgroup (grid_cap
    // is 16 workgroups per CU: below 2 per CU, take one group per thread).
    const int64_t g2 = (n4 + 2 * kPushBlock - 1) / (2 * kPushBlock);
    const bool two = g2 >= (int64_t)grid_cap / 8;
    int64_t grid = two ? g2 : (n4 + kPushBlock - 1) / kPushBlock;
    if (grid > grid_cap) grid = grid_cap;
    if (grid < 1) grid = 1;
    const double inv_hr = 1.0 / ma.hr;
    const dim3 g((unsigned)grid), b(kPushBlock);
    if (push) {
        if (two)
            return dispatch(push_poisson_kernel<true, 2>, g, b, lds, st, zR, zV, n, sub,
                            endrot_tab, endrot_val, K, inv_hr, ma);
        return dispatch(push_poisson_kernel<true, 1>, g, b, lds, st, zR, zV, n, sub, endrot_tab,
                        endrot_val, K, inv_hr, ma);
    }
    if (two)
        return dispatch(push_poisson_kernel<false, 2>, g, b, lds, st, zR, zV, n, sub, endrot_tab,
                        endrot_val, 0, inv_hr, ma);
    return dispatch(push_poisson_kernel<false, 1>, g, b, lds, st, zR, zV, n, sub, endrot_tab,
                    endrot_val, 0, inv_hr, ma);
}

size_t push_lds_bytes_for(int nr) { return push_lds_bytes(nr); }

template <bool P, int U>
static hipError_t raise_lds(int lds)
{
    return raise_dynamic_lds(reinterpret_cast<const void *>(&push_poisson_kernel<P, U>), lds);
}

hipError_t setup_mesh_lds(int nr)
{
    const int lds = (int)push_lds_bytes(nr);
    hipError_t e;
    if ((e = raise_lds<true, 1>(lds)) != hipSuccess) return e;
    if ((e = raise_lds<true, 2>(lds)) != hipSuccess) return e;
    if ((e = raise_lds<false, 1>(lds)) != hipSuccess) return e;
    if ((e = raise_lds<false, 2>(lds)) != hipSuccess) return e;
    for (const void *k : {reinterpret_cast<const void *>(&mesh_solve_kernel<true>),
                          reinterpret_cast<const void *>(&mesh_solve_kernel<false>),
                          reinterpret_cast<const void *>(&potential_kernel)})
        if ((e = raise_dynamic_lds(k, (int)mesh_lds_bytes(nr))) != hipSuccess)
            return e;
    return hipSuccess;
}

// ------------------------------------------------------------ moments

// Per-block FP64 partial sums (fixed-order tree), then one block adds the
// partials in index order: results depend only on n and the grid.
__global__ __launch_bounds__(kMomentBlock) void moments_kernel(
    const float *__restrict__ zR, const float *__restrict__ zV, int64_t n, double c, double s,
    double rmax, double *__restrict__ partial, unsigned long long *__restrict__ pcount)
{
    __shared__ double sd[kMomentBlock];
    __shared__ unsigned long long su[kMomentBlock];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    unsigned long long off = 0ull, bad = 0ull;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
        const double r = zR[i], v = zV[i];
        if (!isfinite(r) || !isfinite(v)) {
            ++bad;
            continue;
        }
        const double R = c * r + s * v;
        const double R2 = R * R;
        a0 += R2;
        a1 += r * r + v * v;
        a2 += R2 * R2;
        if (!(R >= -rmax && R < rmax)) ++off;
    }
    a0 = block_sum<double>(a0, sd);
    a1 = block_sum<double>(a1, sd);
    a2 = block_sum<double>(a2, sd);
    off = block_sum<unsigned long long>(off, su);
    bad = block_sum<unsigned long long>(bad, su);
    if (threadIdx.x == 0) {
        double *p = partial + (size_t)blockIdx.x * kMomentQuantities;
        p[0] = a0;
        p[1] = a1;
        p[2] = a2;
        p[3] = 0.0;
        pcount[(size_t)blockIdx.x * kMomentCounts + 0] = off;
        pcount[(size_t)blockIdx.x * kMomentCounts + 1] = bad;
    }
}

__global__ __launch_bounds__(kMomentBlock) void moments_final_kernel(
    const double *__restrict__ partial, const unsigned long long *__restrict__ pcount, int G,
    double *__restrict__ out, unsigned long long *__restrict__ out_count)
{
    __shared__ double sd[kMomentBlock];
    __shared__ unsigned long long su[kMomentBlock];
    for (int q = 0; q < kMomentQuantities; ++q) {
        double a = 0.0;
        for (int b = threadIdx.x; b < G; b += blockDim.x) a += partial[(size_t)b * kMomentQuantities + q];
        a = block_sum<double>(a, sd);
        if (threadIdx.x == 0) out[q] = a;
    }
    for (int q = 0; q < kMomentCounts; ++q) {
        unsigned long long a = 0ull;
        for (int b = threadIdx.x; b < G; b += blockDim.x) a += pcount[(size_t)b * kMomentCounts + q];
        a = block_sum<unsigned long long>(a, su);
        if (threadIdx.x == 0) out_count[q] = a;
    }
}

int moments_grid(int64_t n)
{
    int64_t g = (n + kMomentBlock - 1) / kMomentBlock;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_moments(hipStream_t st, const float *zR, const float *zV, int64_t n,
                          double c, double s, double rmax, double *partial,
                          unsigned long long *pcount, int grid, double *out,
                          unsigned long long *out_count)
{
    moments_kernel<<<dim3(grid), dim3(kMomentBlock), 0, st>>>(zR, zV, n, c, s, rmax, partial,
                                                              pcount);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    moments_final_kernel<<<dim3(1), dim3(kMomentBlock), 0, st>>>(partial, pcount, grid, out,
                                                                 out_count);
    return hipGetLastError();
}

}  // namespace etd
