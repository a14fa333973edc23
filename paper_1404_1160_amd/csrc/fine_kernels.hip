// HIP kernels of the paper's own solvers (gfx950).
//
// Reference solver: classic RK4 on the characteristics of eq. 1.4,
//   y' = (1/eps) M y + (0, E(t, R)),  M = [[0, 1], [-1, 0]],
// in FP64 in the lab frame.  For the Duffing field every particle is
// independent and one thread runs its whole solve in registers.  For the
// self-consistent field the particles advance in lock step: each RK4 stage is
// one pass over the particles (gather at the stage positions, stage update,
// fixed-point CIC deposit of the next stage positions) followed by the mesh
// solve, so the field is re-solved at every stage as the reference requires.
//
// Improved ETD scheme (Algorithm 3.4), one macro step dt:
//   periods  T_i from the first and third sign change of V along a fine solve
//            from y_i^n (Remark 3.5; the crossing time by linear
//            interpolation of V between fine levels);
//   split    dt = N_i T_i + o_i, 0 <= o_i < T_i;
//   capture  y_i(t_n + o_i) and y_i(t_n + o_i + T_i) from a second fine solve
//            from y_i^n, by quadratic interpolation through the fine levels
//            j-1, j, j+1 around the level j nearest to the time (Remark 3.6);
//   combine  y_i^{n+1} = y_i(o_i) + N_i (y_i(o_i + T_i) - y_i(o_i))  (Lemma 3.3).
// A particle whose velocity has not changed sign three times within max_fine
// fine steps keeps the free period 2 pi eps.

#include "pic_device.h"

namespace etd {

// ------------------------------------------------------------ helpers

__device__ __forceinline__ double quad_interp(double a, double b, double c, double u)
{
    return a * (0.5 * u * (u - 1.0)) + b * (1.0 - u * u) + c * (0.5 * u * (u + 1.0));
}

__device__ __forceinline__ long long near_level(double tau, double inv_h)
{
    const long long j = (long long)floor(tau * inv_h + 0.5);
    return j < 1 ? 1 : j;
}

// whole number of periods and remainder: dt = N T + o, 0 <= o < T
__device__ __forceinline__ void split_step(double dt, double T, long long &N, double &o)
{
    double q = floor(dt / T);
    double r = dt - q * T;
    if (r < 0.0) {
        q -= 1.0;
        r += T;
    }
    if (r >= T) {
        q += 1.0;
        r -= T;
    }
    N = (long long)q;
    o = r;
}

__device__ __forceinline__ void rk4_duffing(double &R, double &V, double h, double ie)
{
    const double k1R = V * ie, k1V = -R * ie - R * R * R;
    double sR = fma(0.5 * h, k1R, R), sV = fma(0.5 * h, k1V, V);
    const double k2R = sV * ie, k2V = -sR * ie - sR * sR * sR;
    sR = fma(0.5 * h, k2R, R);
    sV = fma(0.5 * h, k2V, V);
    const double k3R = sV * ie, k3V = -sR * ie - sR * sR * sR;
    sR = fma(h, k3R, R);
    sV = fma(h, k3V, V);
    const double k4R = sV * ie, k4V = -sR * ie - sR * sR * sR;
    R = fma(h / 6.0, k1R + 2.0 * k2R + 2.0 * k3R + k4R, R);
    V = fma(h / 6.0, k1V + 2.0 * k2V + 2.0 * k3V + k4V, V);
}

// ------------------------------------------------------------ Duffing (per particle)

// Reference RK4: steps of size h, state in FP64 registers; z in the rotating
// frame, y = r(Phi) z with rot0 = (cos, sin) of the start phase and rot1 of
// the end phase.
__global__ __launch_bounds__(256) void rk4_duffing_kernel(float *__restrict__ zR,
                                                          float *__restrict__ zV, int64_t n,
                                                          double h, double ie, long long steps,
                                                          double2 rot0, double2 rot1)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double zr = zR[i], zv = zV[i];
    double R = fma(rot0.x, zr, rot0.y * zv), V = fma(-rot0.y, zr, rot0.x * zv);
    for (long long k = 0; k < steps; ++k) rk4_duffing(R, V, h, ie);
    zR[i] = (float)fma(rot1.x, R, -rot1.y * V);
    zV[i] = (float)fma(rot1.y, R, rot1.x * V);
}

// Improved ETD step for the Duffing field, one particle per thread.  With
// reuse set, T[i] holds the particle's period from an earlier search (in the
// given field each particle's period is constant, section 3) and the search
// is skipped; otherwise the search writes T[i].
__global__ __launch_bounds__(256) void ietd_duffing_kernel(
    float *__restrict__ zR, float *__restrict__ zV, int64_t n, double dt, double h, double ie,
    long long max_fine, double T_free, double2 rot0, double2 rot1, int reuse,
    double *__restrict__ Tio, long long *__restrict__ Nout,
    unsigned long long *__restrict__ unresolved)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double zr = zR[i], zv = zV[i];
    const double R0 = fma(rot0.x, zr, rot0.y * zv), V0 = fma(-rot0.y, zr, rot0.x * zv);
    const double inv_h = 1.0 / h;
    double R = R0, V = V0, T = T_free;
    if (reuse) {
        T = Tio[i];
    } else {
        double t1 = 0.0;
        int cnt = 0;
        for (long long k = 0; k < max_fine && cnt < 3; ++k) {
            const double Vp = V;
            rk4_duffing(R, V, h, ie);
            if ((Vp < 0.0) != (V < 0.0)) {
                const double ts = (double)k * h + h * Vp / (Vp - V);
                if (++cnt == 1) t1 = ts;
                if (cnt == 3) T = ts - t1;
            }
        }
        if (cnt < 3) atomicAdd(unresolved, 1ull);
    }
    if (!(T > 0.0 && T < 1e300)) T = T_free;   // keeps the capture loop bounded
    long long N;
    double o;
    split_step(dt, T, N, o);
    const double tb = o + T;
    const long long ja = near_level(o, inv_h), jb = near_level(tb, inv_h);
    // second solve from y^n with the two captures
    double Rm2 = R0, Vm2 = V0, Rm1 = R0, Vm1 = V0;
    R = R0;
    V = V0;
    double Ra = R0, Va = V0, Rb = R0, Vb = V0;
    for (long long L = 1; L <= jb + 1; ++L) {
        Rm2 = Rm1;
        Vm2 = Vm1;
        Rm1 = R;
        Vm1 = V;
        rk4_duffing(R, V, h, ie);
        if (L < 2) continue;
        if (ja + 1 == L) {
            const double u = (o - (double)ja * h) * inv_h;
            Ra = quad_interp(Rm2, Rm1, R, u);
            Va = quad_interp(Vm2, Vm1, V, u);
        }
        if (jb + 1 == L) {
            const double u = (tb - (double)jb * h) * inv_h;
            Rb = quad_interp(Rm2, Rm1, R, u);
            Vb = quad_interp(Vm2, Vm1, V, u);
        }
    }
    const double q = (double)N;
    const double R1 = fma(q, Rb - Ra, Ra), V1 = fma(q, Vb - Va, Va);
    zR[i] = (float)fma(rot1.x, R1, -rot1.y * V1);
    zV[i] = (float)fma(rot1.y, R1, rot1.x * V1);
    if (!reuse) Tio[i] = T;
    Nout[i] = N;
}

hipError_t launch_rk4_duffing(hipStream_t st, float *zR, float *zV, int64_t n, double h,
                              double eps, long long steps, double2 rot0, double2 rot1)
{
    if (n <= 0) return hipSuccess;
    return dispatch(rk4_duffing_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, zR,
                    zV, n, h, 1.0 / eps, steps, rot0, rot1);
}

hipError_t launch_ietd_duffing(hipStream_t st, float *zR, float *zV, int64_t n, double dt,
                               double h, double eps, long long max_fine, double2 rot0,
                               double2 rot1, bool reuse, double *T, long long *N,
                               unsigned long long *unresolved)
{
    if (n <= 0) return hipSuccess;
    return dispatch(ietd_duffing_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, zR,
                    zV, n, dt, h, 1.0 / eps, max_fine, 2.0 * 3.141592653589793 * eps, rot0, rot1,
                    reuse ? 1 : 0, T, N, unresolved);
}

// Periods only (the modified ETD scheme needs their mean first).
__global__ __launch_bounds__(256) void period_duffing_kernel(
    const float *__restrict__ zR, const float *__restrict__ zV, int64_t n, double h, double ie,
    long long max_fine, double T_free, double2 rot0, double *__restrict__ Tout,
    unsigned long long *__restrict__ unresolved)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double zr = zR[i], zv = zV[i];
    double R = fma(rot0.x, zr, rot0.y * zv), V = fma(-rot0.y, zr, rot0.x * zv);
    double t1 = 0.0, T = T_free;
    int cnt = 0;
    for (long long k = 0; k < max_fine && cnt < 3; ++k) {
        const double Vp = V;
        rk4_duffing(R, V, h, ie);
        if ((Vp < 0.0) != (V < 0.0)) {
            const double ts = (double)k * h + h * Vp / (Vp - V);
            if (++cnt == 1) t1 = ts;
            if (cnt == 3) T = ts - t1;
        }
    }
    if (cnt < 3) atomicAdd(unresolved, 1ull);
    Tout[i] = T;
}

// Classic ETD step (Algorithm 2.1) with the common period P = dt - N o:
// K1 equal steps over P give y(t_n + P); y(t_n + N P) = y^n + N (y(t_n + P)
// - y^n); K2 equal steps over o give y^{n+1}.
__global__ __launch_bounds__(256) void cetd_duffing_kernel(float *__restrict__ zR,
                                                           float *__restrict__ zV, int64_t n,
                                                           double hP, long long K1, double ho,
                                                           long long K2, double q, double ie,
                                                           double2 rot0, double2 rot1)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double zr = zR[i], zv = zV[i];
    const double R0 = fma(rot0.x, zr, rot0.y * zv), V0 = fma(-rot0.y, zr, rot0.x * zv);
    double R = R0, V = V0;
    for (long long k = 0; k < K1; ++k) rk4_duffing(R, V, hP, ie);
    R = fma(q, R - R0, R0);
    V = fma(q, V - V0, V0);
    for (long long k = 0; k < K2; ++k) rk4_duffing(R, V, ho, ie);
    zR[i] = (float)fma(rot1.x, R, -rot1.y * V);
    zV[i] = (float)fma(rot1.y, R, rot1.x * V);
}

// Sum of x[0..n) in a fixed order: per-block partial sums (strided per
// thread, then the block's fixed-order tree), then one block adds the
// partials in index order.
__global__ __launch_bounds__(256) void sum_partial_kernel(const double *__restrict__ x, int64_t n,
                                                          double *__restrict__ partial)
{
    __shared__ double wt[4];
    double a = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a += x[i];
    a = block_sum<double>(a, wt);
    if (threadIdx.x == 0) partial[blockIdx.x] = a;
}

__global__ __launch_bounds__(256) void sum_final_kernel(const double *__restrict__ partial, int g,
                                                        double *__restrict__ out)
{
    __shared__ double wt[4];
    double a = 0.0;
    for (int i = threadIdx.x; i < g; i += blockDim.x) a += partial[i];
    a = block_sum<double>(a, wt);
    if (threadIdx.x == 0) *out = a;
}

__global__ __launch_bounds__(256) void fill_ll_kernel(long long *__restrict__ x, int64_t n,
                                                      long long v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

hipError_t launch_period_duffing(hipStream_t st, const float *zR, const float *zV, int64_t n,
                                 double h, double eps, long long max_fine, double2 rot0, double *T,
                                 unsigned long long *unresolved)
{
    if (n <= 0) return hipSuccess;
    return dispatch(period_duffing_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, zR,
                    zV, n, h, 1.0 / eps, max_fine, 2.0 * 3.141592653589793 * eps, rot0, T,
                    unresolved);
}

hipError_t launch_cetd_duffing(hipStream_t st, float *zR, float *zV, int64_t n, double hP,
                               long long K1, double ho, long long K2, double q, double eps,
                               double2 rot0, double2 rot1)
{
    if (n <= 0) return hipSuccess;
    return dispatch(cetd_duffing_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, zR,
                    zV, n, hP, K1, ho, K2, q, 1.0 / eps, rot0, rot1);
}

hipError_t launch_sum(hipStream_t st, const double *x, int64_t n, double *partial, int g,
                      double *out)
{
    sum_partial_kernel<<<dim3((unsigned)g), dim3(256), 0, st>>>(x, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    sum_final_kernel<<<dim3(1), dim3(256), 0, st>>>(partial, g, out);
    return hipGetLastError();
}

hipError_t launch_fill_ll(hipStream_t st, long long *x, int64_t n, long long v)
{
    if (n <= 0) return hipSuccess;
    fill_ll_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(x, n, v);
    return hipGetLastError();
}

// ------------------------------------------------------------ Poisson (lock step)

// Stage kernel of the coupled RK4 step from level L-1 to level L (t = L h).
// Stage 1 evaluates at y, stages 2-4 at the stage state s; the field in etab
// is the one of the positions being evaluated.  Stages 1-3 deposit the next
// stage positions, stage 4 deposits y_L.  MODE 1 (period search) and MODE 2
// (captures) do their bookkeeping in stage 4.
template <int STAGE, int MODE>
__global__ __launch_bounds__(kPushBlock) void rk4_stage_kernel(FineArgs a, int64_t n, double h,
                                                              double ie, long long L,
                                                              double inv_hr, MeshArgs ma)
{
    const int nr = ma.nr;
    extern __shared__ __align__(16) unsigned char smem[];
    float2 *Et = reinterpret_cast<float2 *>(smem);
    unsigned long long *H =
        reinterpret_cast<unsigned long long *>(smem + (size_t)nr * sizeof(float2));
    const int tid = threadIdx.x;
    for (int k = tid; k < nr; k += blockDim.x) Et[k] = ma.etab[k];
    for (int k = tid; k <= nr; k += blockDim.x) H[k] = 0ull;
    MeshView m;
    m.Et = Et;
    m.H = H;
    m.inv_hr = inv_hr;
    m.half = 0.5 * (double)nr;
    m.c = nr >> 1;
    m.Qb = ma.fscal[kQb];
    unsigned done = 0u;
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + tid; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double yR = a.yR[i], yV = a.yV[i];
        const double pR = STAGE == 1 ? yR : a.sR[i], pV = STAGE == 1 ? yV : a.sV[i];
        const double kR = pV * ie, kV = fma(-pR, ie, gather(m, pR));
        if (STAGE < 4) {
            double accR, accV;
            if (STAGE == 1) {
                accR = kR;
                accV = kV;
            } else {
                accR = fma(2.0, kR, a.aR[i]);
                accV = fma(2.0, kV, a.aV[i]);
            }
            a.aR[i] = accR;
            a.aV[i] = accV;
            const double c = STAGE == 3 ? h : 0.5 * h;
            const double nR = fma(c, kR, yR), nV = fma(c, kV, yV);
            a.sR[i] = nR;
            a.sV[i] = nV;
            deposit(m, nR);
        } else {
            const double R = fma(h / 6.0, a.aR[i] + kR, yR);
            const double V = fma(h / 6.0, a.aV[i] + kV, yV);
            if (MODE == 1 && a.cnt[i] < 3 && (yV < 0.0) != (V < 0.0)) {
                const double ts = (double)(L - 1) * h + h * yV / (yV - V);
                const int c = a.cnt[i] + 1;
                a.cnt[i] = c;
                if (c == 1) a.t1[i] = ts;
                if (c == 3) {
                    a.T[i] = ts - a.t1[i];
                    ++done;
                }
            }
            if (MODE == 2) {
                // levels L-2 (stored), L-1 (= y) and L
                const double inv_h = 1.0 / h;
                const double pR2 = a.pR[i], pV2 = a.pV[i];
                if (L >= 2) {
                    const double o = a.o[i], tb = o + a.T[i];
                    const long long ja = near_level(o, inv_h), jb = near_level(tb, inv_h);
                    if (ja + 1 == L) {
                        const double u = (o - (double)ja * h) * inv_h;
                        a.cR[i] = quad_interp(pR2, yR, R, u);
                        a.cV[i] = quad_interp(pV2, yV, V, u);
                    }
                    if (jb + 1 == L) {
                        const double u = (tb - (double)jb * h) * inv_h;
                        a.dR[i] = quad_interp(pR2, yR, R, u);
                        a.dV[i] = quad_interp(pV2, yV, V, u);
                    }
                }
                a.pR[i] = yR;
                a.pV[i] = yV;
            }
            a.yR[i] = R;
            a.yV[i] = V;
            deposit(m, R);
        }
    }
    if (MODE == 1 && STAGE == 4) {
        // particles that found their third sign change: wave sums, one atomic
        // per wave
        unsigned long long d = wave_sum<unsigned long long>((unsigned long long)done);
        if ((tid & 63) == 0 && d) atomicAdd(a.done, d);
    }
    __syncthreads();
    const int nn = nr + 1;
    const int start = (int)(((unsigned)blockIdx.x * 131u) % (unsigned)nn);
    for (int k0 = tid; k0 < nn; k0 += blockDim.x) {
        int k = k0 + start;
        if (k >= nn) k -= nn;
        const unsigned long long v = H[k];
        if (v) atomicAdd(&ma.hist[k], v);
    }
}

// Deposit of the FP64 lab-frame positions yR (field of the start level).
__global__ __launch_bounds__(kPushBlock) void fine_deposit_kernel(const double *__restrict__ yR,
                                                                 int64_t n, double inv_hr,
                                                                 MeshArgs ma)
{
    const int nr = ma.nr;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long *H = reinterpret_cast<unsigned long long *>(smem);
    const int tid = threadIdx.x;
    for (int k = tid; k <= nr; k += blockDim.x) H[k] = 0ull;
    MeshView m;
    m.Et = nullptr;
    m.H = H;
    m.inv_hr = inv_hr;
    m.half = 0.5 * (double)nr;
    m.c = nr >> 1;
    m.Qb = 0.0;
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + tid; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        deposit(m, yR[i]);
    __syncthreads();
    const int nn = nr + 1;
    const int start = (int)(((unsigned)blockIdx.x * 131u) % (unsigned)nn);
    for (int k0 = tid; k0 < nn; k0 += blockDim.x) {
        int k = k0 + start;
        if (k >= nn) k -= nn;
        const unsigned long long v = H[k];
        if (v) atomicAdd(&ma.hist[k], v);
    }
}

// Start of a fine solve: y = y0 = r(Phi_n) z (and the level L-2 store); for a
// period search, the counters are cleared.
__global__ __launch_bounds__(256) void fine_begin_kernel(FineArgs a, const float *__restrict__ zR,
                                                        const float *__restrict__ zV, int64_t n,
                                                        double2 rot0, int mode, double T_free)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double zr = zR[i], zv = zV[i];
    const double R = fma(rot0.x, zr, rot0.y * zv), V = fma(-rot0.y, zr, rot0.x * zv);
    a.yR[i] = R;
    a.yV[i] = V;
    if (mode == 1) {
        a.cnt[i] = 0;
        a.T[i] = T_free;
    }
    if (mode == 3) {   // classic ETD: keep y^n
        a.pR[i] = R;
        a.pV[i] = V;
    }
    if (mode == 2) {
        a.pR[i] = R;
        a.pV[i] = V;
        a.cR[i] = R;
        a.cV[i] = V;
        a.dR[i] = R;
        a.dV[i] = V;
    }
}

// Classic ETD, step 2: y(t_n + N P) = y^n + N (y(t_n + P) - y^n), y^n in p.
__global__ __launch_bounds__(256) void cetd_combine_kernel(FineArgs a, int64_t n, double q)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double R0 = a.pR[i], V0 = a.pV[i];
    a.yR[i] = fma(q, a.yR[i] - R0, R0);
    a.yV[i] = fma(q, a.yV[i] - V0, V0);
}

hipError_t launch_cetd_combine(hipStream_t st, const FineArgs &a, int64_t n, double q)
{
    if (n <= 0) return hipSuccess;
    cetd_combine_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(a, n, q);
    return hipGetLastError();
}

// After the period search: split dt, and the last fine level the captures need.
__global__ __launch_bounds__(256) void ietd_split_kernel(FineArgs a, int64_t n, double dt, double h)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    unsigned long long last = 0ull, unres = 0ull;
    if (i < n) {
        long long N;
        double o;
        split_step(dt, a.T[i], N, o);
        a.N[i] = N;
        a.o[i] = o;
        last = (unsigned long long)(near_level(o + a.T[i], 1.0 / h) + 1);
        unres = a.cnt[i] < 3 ? 1ull : 0ull;
    }
    // wave maxima / sums, one atomic each per wave
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long u = __shfl_xor(last, off, 64);
        last = u > last ? u : last;
    }
    unres = wave_sum<unsigned long long>(unres);
    if ((threadIdx.x & 63) == 0) {
        atomicMax(a.last, last);
        if (unres) atomicAdd(a.unresolved, unres);
    }
}

// End of a macro step: y^{n+1} (improved ETD: from the captures; reference:
// the fine state) to the rotating frame at Phi_{n+1}.
__global__ __launch_bounds__(256) void fine_end_kernel(FineArgs a, float *__restrict__ zR,
                                                      float *__restrict__ zV, int64_t n,
                                                      double2 rot1, int ietd)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double R, V;
    if (ietd) {
        const double q = (double)a.N[i];
        R = fma(q, a.dR[i] - a.cR[i], a.cR[i]);
        V = fma(q, a.dV[i] - a.cV[i], a.cV[i]);
    } else {
        R = a.yR[i];
        V = a.yV[i];
    }
    zR[i] = (float)fma(rot1.x, R, -rot1.y * V);
    zV[i] = (float)fma(rot1.y, R, rot1.x * V);
}

static size_t stage_lds_bytes(int nr)
{
    return (size_t)nr * sizeof(float2) + (size_t)(nr + 1) * sizeof(unsigned long long);
}

template <int S, int M>
static hipError_t launch_stage_t(hipStream_t st, const FineArgs &a, int64_t n, double h,
                                 double eps, long long L, const MeshArgs &ma, int grid)
{
    return dispatch(rk4_stage_kernel<S, M>, dim3((unsigned)grid), dim3(kPushBlock),
                    stage_lds_bytes(ma.nr), st, a, n, h, 1.0 / eps, L, 1.0 / ma.hr, ma);
}

static int fine_grid(int64_t n, int cap)
{
    int64_t g = (n + kPushBlock - 1) / kPushBlock;
    if (g > cap) g = cap;
    return g < 1 ? 1 : (int)g;
}

hipError_t launch_rk4_stage(hipStream_t st, int stage, int mode, const FineArgs &a, int64_t n,
                            double h, double eps, long long L, const MeshArgs &ma, int grid_cap)
{
    if (n <= 0) return hipSuccess;
    const int g = fine_grid(n, grid_cap);
#define ETD_STAGE(S, M)                                                                       \
    if (stage == S && mode == M) return launch_stage_t<S, M>(st, a, n, h, eps, L, ma, g);
    ETD_STAGE(1, 0) ETD_STAGE(2, 0) ETD_STAGE(3, 0) ETD_STAGE(4, 0)
    ETD_STAGE(1, 1) ETD_STAGE(2, 1) ETD_STAGE(3, 1) ETD_STAGE(4, 1)
    ETD_STAGE(1, 2) ETD_STAGE(2, 2) ETD_STAGE(3, 2) ETD_STAGE(4, 2)
#undef ETD_STAGE
    return hipErrorInvalidValue;
}

hipError_t launch_fine_deposit(hipStream_t st, const double *yR, int64_t n, const MeshArgs &ma,
                               int grid_cap)
{
    if (n <= 0) return hipSuccess;
    return dispatch(fine_deposit_kernel, dim3((unsigned)fine_grid(n, grid_cap)), dim3(kPushBlock),
                    (size_t)(ma.nr + 1) * sizeof(unsigned long long), st, yR, n, 1.0 / ma.hr, ma);
}

hipError_t launch_fine_begin(hipStream_t st, const FineArgs &a, const float *zR, const float *zV,
                             int64_t n, double2 rot0, int mode, double eps)
{
    if (n <= 0) return hipSuccess;
    return dispatch(fine_begin_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, zR,
                    zV, n, rot0, mode, 2.0 * 3.141592653589793 * eps);
}

hipError_t launch_ietd_split(hipStream_t st, const FineArgs &a, int64_t n, double dt, double h)
{
    if (n <= 0) return hipSuccess;
    return dispatch(ietd_split_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n,
                    dt, h);
}

hipError_t launch_fine_end(hipStream_t st, const FineArgs &a, float *zR, float *zV, int64_t n,
                           double2 rot1, int ietd)
{
    if (n <= 0) return hipSuccess;
    return dispatch(fine_end_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, zR, zV,
                    n, rot1, ietd);
}

hipError_t setup_fine_lds(int nr)
{
    hipError_t e;
#define ETD_LDS(S, M)                                                                           \
    e = raise_dynamic_lds(reinterpret_cast<const void *>(&rk4_stage_kernel<S, M>),             \
                          (int)stage_lds_bytes(nr));                                            \
    if (e != hipSuccess) return e;
    ETD_LDS(1, 0) ETD_LDS(2, 0) ETD_LDS(3, 0) ETD_LDS(4, 0)
    ETD_LDS(1, 1) ETD_LDS(2, 1) ETD_LDS(3, 1) ETD_LDS(4, 1)
    ETD_LDS(1, 2) ETD_LDS(2, 2) ETD_LDS(3, 2) ETD_LDS(4, 2)
#undef ETD_LDS
    return raise_dynamic_lds(reinterpret_cast<const void *>(&fine_deposit_kernel),
                             (int)((nr + 1) * sizeof(unsigned long long)));
}

}  // namespace etd
