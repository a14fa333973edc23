// Device functions of the plain push shared by the fused push+deposit kernel
// and the sorted-deposit kernels: the frozen-field CIC gather, the fixed-point
// CIC deposit and the K-substep midpoint push in the rotating frame.
#pragma once

#include "internal.h"

namespace etd {

constexpr double kFixOne = 4294967296.0;              // 2^32
constexpr double kFixScale = 2.3283064365386963e-10;  // 2^-32

// Cell of a lab-frame position: on the mesh iff -half <= R/h_r < half; then
// node k = floor(R/h_r) + nr/2 and th = R/h_r - floor(R/h_r) in [0, 1).
__device__ __forceinline__ bool cell_of(double R, double inv_hr, double half, int c, int &k,
                                        double &th)
{
    const double x = R * inv_hr;
    if (!(x >= -half && x < half)) return false;
    const double fl = floor(x);
    th = x - fl;
    k = (int)fl + c;
    return true;
}

__device__ __forceinline__ unsigned int fixed_weight(double th)
{
    return (unsigned int)(th * kFixOne);
}

struct MeshView {
    const float2 *Et;       // LDS: (E_m, E_{m+1} - E_m), m = 0..nr-1
    unsigned long long *H;  // LDS: fixed-point node charges, nr+1
    double inv_hr;
    double half;            // nr/2: on-mesh iff -half <= R/h_r < half
    int c;                  // centre node
    double Qb;              // half enclosed charge at the edge
};

// CIC gather of the frozen field at R; off the mesh (and for NaN) E = Qb / R.
__device__ __forceinline__ double gather(const MeshView &m, double R)
{
    int k;
    double th;
    if (cell_of(R, m.inv_hr, m.half, m.c, k, th)) {
        const float2 e = m.Et[k];
        return fma(th, (double)e.y, (double)e.x);
    }
    return m.Qb / R;
}

// The gather of a position known to lie on the mesh: the arithmetic of
// gather() without its range test, so the same bits for such R.  Without the
// branch the compiler can keep several particles' table reads in flight.
__device__ __forceinline__ double gather_on(const MeshView &m, double R)
{
    const double x = R * m.inv_hr;
    const double fl = floor(x);
    const float2 e = m.Et[(int)fl + m.c];
    return fma(x - fl, (double)e.y, (double)e.x);
}

// A particle with |z|^2 below this value stays on the mesh at every substep
// position of a K-substep push: R_mid = (cos, sin) . (z + a) with |a| at most
// the sum of the Duhamel increments h |E| <= K h emax (by induction, since
// every earlier position was on the mesh).  The margin 1e-9 covers the FP64
// rounding of R_mid and R / h_r.  Negative when no |z| qualifies.
__device__ __forceinline__ double on_mesh_limit2(const MeshView &m, const double4 *sub, int K,
                                                 double emax)
{
    const double4 q = sub[0];
    const double reach = (double)K * sqrt(q.z * q.z + q.w * q.w) * emax;
    const double lim = m.half / m.inv_hr * (1.0 - 1e-9) - reach;
    return lim > 0.0 ? lim * lim : -1.0;
}

// CIC deposit of one particle at R into the LDS histogram (skipped off-mesh):
// weights 1 - th and th in units of 2^-32 of a particle weight.
__device__ __forceinline__ void deposit(const MeshView &m, double R)
{
    int k;
    double th;
    if (cell_of(R, m.inv_hr, m.half, m.c, k, th)) {
        const unsigned int q = fixed_weight(th);
        atomicAdd(&m.H[k], (unsigned long long)(4294967296ull - q));
        atomicAdd(&m.H[k + 1], (unsigned long long)q);
    }
}

// K substeps of NP particles in the frozen field; ON: every substep
// position is known to lie on the mesh (on_mesh_limit2).  The ON loop does
// the arithmetic of gather_on in three phases (cell positions of all NP
// particles, their table reads, then the updates), so that the NP reads are
// in flight together, and reads the next substep's coefficients ahead; same
// results as the general loop.
template <int NP, bool ON = false>
__device__ __forceinline__ void push_group(const MeshView &m, const double4 *__restrict__ sub,
                                           int K, double (&zr)[NP], double (&zv)[NP])
{
    double ar[NP], av[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) ar[p] = av[p] = 0.0;
    if (ON) {
        double4 q = sub[0];
        for (int k = 0; k < K; ++k) {
            const double4 qn = sub[k + 1 < K ? k + 1 : k];
            double x[NP], fl[NP];
            float2 e[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                x[p] = fma(q.x, zr[p] + ar[p], q.y * (zv[p] + av[p])) * m.inv_hr;
                fl[p] = floor(x[p]);
            }
#pragma unroll
            for (int p = 0; p < NP; ++p) e[p] = m.Et[(int)fl[p] + m.c];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const double E = fma(x[p] - fl[p], (double)e[p].y, (double)e[p].x);
                ar[p] = fma(-q.z, E, ar[p]);
                av[p] = fma(q.w, E, av[p]);
            }
            q = qn;
        }
    } else {
        for (int k = 0; k < K; ++k) {
            const double4 q = sub[k];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const double Rm = fma(q.x, zr[p] + ar[p], q.y * (zv[p] + av[p]));
                const double E = gather(m, Rm);
                ar[p] = fma(-q.z, E, ar[p]);
                av[p] = fma(q.w, E, av[p]);
            }
        }
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        zr[p] += ar[p];
        zv[p] += av[p];
    }
}


// Wave (64-lane) and block scans and sums with a fixed combination order, so
// FP64 results are reproducible run to run.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Exclusive prefix of v over the block (wtot: LDS scratch of >= 16 entries).
template <typename T>
__device__ T block_exclusive_scan(T v, T *wtot)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const T incl = wave_inclusive_scan(v);
    T excl = __shfl_up(incl, 1, 64);
    if (lane == 0) excl = T(0);
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    if (w == 0) {
        const T t = lane < nw ? wtot[lane] : T(0);
        const T ti = wave_inclusive_scan(t);
        T te = __shfl_up(ti, 1, 64);
        if (lane == 0) te = T(0);
        if (lane < nw) wtot[lane] = te;
    }
    __syncthreads();
    const T r = wtot[w] + excl;
    __syncthreads();
    return r;
}

template <typename T>
__device__ T block_sum(T v, T *wtot)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    if (lane == 0) wtot[w] = v;
    __syncthreads();
    T r = T(0);
    for (int i = 0; i < nw; ++i) r += wtot[i];
    __syncthreads();
    return r;
}

}  // namespace etd
