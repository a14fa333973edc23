// Deterministic sort-by-cell CIC deposit (gfx950).
//
// Per Poisson step, instead of the fused push + LDS-histogram deposit:
//   sort_count_kernel    push each particle in registers (K substeps, frozen
//                        field) and count the cell keys of the new positions
//                        per workgroup (key nr = off the mesh)
//   sort_offsets_kernel  per key, exclusive offsets of the workgroups' counts
//   sort_starts_kernel   exclusive scan of the key totals: segment starts
//   sort_scatter_kernel  push again (same arithmetic, same keys) and write each
//                        particle, with its id, to its slot in cell order
//   sort_reduce_kernel   one workgroup per cell: segmented reduction of the
//                        CIC weights of that cell's contiguous particles
// The weights are the same 2^-32 fixed-point integers as the fused deposit,
// so the node charges are bitwise identical to it; particles within one
// (workgroup, cell) segment may land in any order, which changes no result.

#include "pic_device.h"

namespace etd {

namespace {

struct SortLds {
    float2 *Et;
    unsigned *C;
};

__device__ __forceinline__ SortLds sort_lds(unsigned char *smem, int nr)
{
    SortLds s;
    s.Et = reinterpret_cast<float2 *>(smem);
    s.C = reinterpret_cast<unsigned *>(smem + (size_t)nr * sizeof(float2));
    return s;
}

// New FP32 state and cell key of one particle after the step.  FAST: a
// particle with |z|^2 < lim2 (see on_mesh_limit2) takes the gather without
// range tests; it pays only for several substeps, so the launchers choose it
// for K > 1.
template <bool FAST>
__device__ __forceinline__ void step_one(const MeshView &m, const double4 *__restrict__ sub, int K,
                                         double lim2, double2 er, float &fr, float &fv, int nr,
                                         int &key)
{
    double zr[1] = {fr}, zv[1] = {fv};
    if (FAST && fma(zr[0], zr[0], zv[0] * zv[0]) < lim2)
        push_group<1, true>(m, sub, K, zr, zv);
    else
        push_group<1>(m, sub, K, zr, zv);
    fr = (float)zr[0];
    fv = (float)zv[0];
    int k;
    double th;
    key = cell_of(fma(er.x, (double)fr, er.y * (double)fv), m.inv_hr, m.half, m.c, k, th) ? k
                                                                                          : nr;
}

}  // namespace

// Both passes visit the particles in the same order (float4 groups with a
// grid stride, then the ragged tail), so that they assign each particle to
// the same workgroup.
template <bool SCATTER, bool FAST>
__global__ __launch_bounds__(kPushBlock) void sort_pass_kernel(
    const float *__restrict__ zR, const float *__restrict__ zV, const unsigned *__restrict__ ids,
    int64_t n, const double4 *__restrict__ sub, const double2 *__restrict__ endrot, int K,
    double inv_hr, const float2 *__restrict__ etab, const double *__restrict__ fscal, int nr,
    unsigned *__restrict__ counts, const unsigned *__restrict__ starts,
    float *__restrict__ oR, float *__restrict__ oV, unsigned *__restrict__ oid)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const SortLds L = sort_lds(smem, nr);
    const int tid = threadIdx.x;
    const int nk = nr + 1;
    unsigned *cnt = counts + (size_t)blockIdx.x * nk;
    for (int i = tid; i < nr; i += blockDim.x) L.Et[i] = etab[i];
    for (int i = tid; i < nk; i += blockDim.x) L.C[i] = SCATTER ? starts[i] + cnt[i] : 0u;
    MeshView m;
    m.Et = L.Et;
    m.H = nullptr;
    m.inv_hr = inv_hr;
    m.half = 0.5 * (double)nr;
    m.c = nr >> 1;
    m.Qb = fscal[kQb];
    const double2 er = endrot[0];
    const double lim2 = FAST ? on_mesh_limit2(m, sub, K, fscal[kEmax]) : -1.0;
    __syncthreads();

    auto visit = [&](int64_t i, float fr, float fv) {
        int key;
        step_one<FAST>(m, sub, K, lim2, er, fr, fv, nr, key);
        const unsigned slot = atomicAdd(&L.C[key], 1u);
        if (SCATTER) {
            oR[slot] = fr;
            oV[slot] = fv;
            oid[slot] = ids[i];
        }
    };
    const int64_t n4 = n >> 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const float4 *zR4 = reinterpret_cast<const float4 *>(zR);
    const float4 *zV4 = reinterpret_cast<const float4 *>(zV);
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + tid; g < n4; g += stride) {
        const float4 r4 = zR4[g], v4 = zV4[g];
        visit(4 * g, r4.x, v4.x);
        visit(4 * g + 1, r4.y, v4.y);
        visit(4 * g + 2, r4.z, v4.z);
        visit(4 * g + 3, r4.w, v4.w);
    }
    const int64_t gt = blockIdx.x * (int64_t)blockDim.x + tid;
    if (gt < n - (n4 << 2)) {
        const int64_t i = (n4 << 2) + gt;
        visit(i, zR[i], zV[i]);
    }
    if (!SCATTER) {
        __syncthreads();
        for (int i = tid; i < nk; i += blockDim.x) cnt[i] = L.C[i];
    }
}

// counts[b][k] <- sum_{b' < b} counts[b'][k];  total[k] = sum_b counts[b][k].
// A workgroup takes 16 keys; its 16 x 16 threads split the G rows of those
// keys into 16 chunks: chunk sums, a scan over the chunks, then the rows.
constexpr int kOffKeys = 16, kOffChunks = 16;

__global__ __launch_bounds__(kOffKeys * kOffChunks) void sort_offsets_kernel(
    unsigned *__restrict__ counts, int G, int nk, unsigned *__restrict__ total)
{
    __shared__ unsigned part[kOffChunks][kOffKeys];
    const int kl = threadIdx.x % kOffKeys, ch = threadIdx.x / kOffKeys;
    const int k = blockIdx.x * kOffKeys + kl;
    const int rows = (G + kOffChunks - 1) / kOffChunks;
    const int b0 = ch * rows, b1 = min(b0 + rows, G);
    unsigned sum = 0;
    if (k < nk)
        for (int b = b0; b < b1; ++b) sum += counts[(size_t)b * nk + k];
    part[ch][kl] = sum;
    __syncthreads();
    if (ch == 0) {
        unsigned run = 0;
        for (int c = 0; c < kOffChunks; ++c) {
            const unsigned v = part[c][kl];
            part[c][kl] = run;
            run += v;
        }
        if (k < nk) total[k] = run;
    }
    __syncthreads();
    if (k < nk) {
        unsigned run = part[ch][kl];
        for (int b = b0; b < b1; ++b) {
            const unsigned v = counts[(size_t)b * nk + k];
            counts[(size_t)b * nk + k] = run;
            run += v;
        }
    }
}

// starts[k] = sum_{k' < k} total[k'] (one workgroup, contiguous chunks)
__global__ __launch_bounds__(1024) void sort_starts_kernel(const unsigned *__restrict__ total,
                                                           int nk, unsigned *__restrict__ starts)
{
    __shared__ unsigned wtot[16];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int chunk = (nk + nt - 1) / nt;
    const int k0 = min(tid * chunk, nk), k1 = min(k0 + chunk, nk);
    unsigned loc = 0;
    for (int k = k0; k < k1; ++k) loc += total[k];
    unsigned run = block_exclusive_scan<unsigned>(loc, wtot);
    for (int k = k0; k < k1; ++k) {
        starts[k] = run;
        run += total[k];
    }
}

// Segmented reduction: one workgroup per cell k.  The cell's particles are
// contiguous in cell order; their weights (1 - th, th) go to nodes k and k+1
// (one wave-tree sum, two global atomics per cell).  Keys are recomputed
// with the arithmetic of the count and scatter passes, so every particle of
// the segment lies in cell k; a particle that did not would be added on its
// own.
__global__ __launch_bounds__(256) void sort_reduce_kernel(
    const float *__restrict__ zR, const float *__restrict__ zV, const unsigned *__restrict__ starts,
    const unsigned *__restrict__ total, const double2 *__restrict__ endrot, double inv_hr, int nr,
    unsigned long long *__restrict__ hist)
{
    __shared__ unsigned long long wtot[4];
    const int k = blockIdx.x;
    const double2 er = endrot[0];
    const double half = 0.5 * (double)nr;
    const int c = nr >> 1;
    const unsigned s0 = starts[k], cnt = total[k];
    unsigned long long A = 0ull, B = 0ull;
    for (unsigned j = threadIdx.x; j < cnt; j += blockDim.x) {
        const unsigned i = s0 + j;
        int kk;
        double th;
        if (cell_of(fma(er.x, (double)zR[i], er.y * (double)zV[i]), inv_hr, half, c, kk, th)) {
            const unsigned q = fixed_weight(th);
            if (kk == k) {
                A += 4294967296ull - q;
                B += q;
            } else {
                atomicAdd(&hist[kk], 4294967296ull - q);
                atomicAdd(&hist[kk + 1], (unsigned long long)q);
            }
        }
    }
    A = block_sum<unsigned long long>(A, wtot);
    B = block_sum<unsigned long long>(B, wtot);
    if (threadIdx.x == 0) {
        if (A) atomicAdd(&hist[k], A);
        if (B) atomicAdd(&hist[k + 1], B);
    }
}

__global__ void iota_kernel(unsigned *__restrict__ ids, int64_t first, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) ids[first + i] = (unsigned)(first + i);
}

__global__ void inverse_kernel(const unsigned *__restrict__ ids, int64_t n,
                               unsigned *__restrict__ inv)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) inv[ids[i]] = (unsigned)i;
}

// y = r(phi) z of particles inv[first + j], j < count (original order)
__global__ void gather_out_kernel(const float *__restrict__ zR, const float *__restrict__ zV,
                                  const unsigned *__restrict__ inv, int64_t first, int64_t count,
                                  double c, double s, double *__restrict__ R,
                                  double *__restrict__ V)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j < count) {
        const unsigned i = inv[first + j];
        const double r = zR[i], v = zV[i];
        R[j] = c * r + s * v;
        V[j] = -s * r + c * v;
    }
}

// z of particles inv[j] in original order j < n (FP32 copies)
__global__ void gather_f32_kernel(const float *__restrict__ zR, const float *__restrict__ zV,
                                  const unsigned *__restrict__ inv, int64_t n,
                                  float *__restrict__ oR, float *__restrict__ oV)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j < n) {
        const unsigned i = inv[j];
        oR[j] = zR[i];
        oV[j] = zV[i];
    }
}

hipError_t launch_gather_f32(hipStream_t st, const float *zR, const float *zV, const unsigned *inv,
                             int64_t n, float *oR, float *oV)
{
    if (n <= 0) return hipSuccess;
    gather_f32_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(zR, zV, inv, n, oR,
                                                                             oV);
    return hipGetLastError();
}

static size_t sort_lds_bytes(int nr)
{
    return (size_t)nr * sizeof(float2) + (size_t)(nr + 1) * sizeof(unsigned);
}

hipError_t setup_sort_lds(int nr)
{
    const int lds = (int)sort_lds_bytes(nr);
    for (const void *f : {reinterpret_cast<const void *>(&sort_pass_kernel<false, false>),
                          reinterpret_cast<const void *>(&sort_pass_kernel<false, true>),
                          reinterpret_cast<const void *>(&sort_pass_kernel<true, false>),
                          reinterpret_cast<const void *>(&sort_pass_kernel<true, true>)}) {
        const hipError_t e = raise_dynamic_lds(f, lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_sort_count(hipStream_t st, const SortArgs &a, int grid)
{
    return dispatch(a.K > 1 ? sort_pass_kernel<false, true> : sort_pass_kernel<false, false>,
                    dim3(grid), dim3(kPushBlock), sort_lds_bytes(a.nr), st, a.zR, a.zV, a.ids,
                    a.n, a.sub, a.endrot, a.K, a.inv_hr, a.etab, a.fscal, a.nr, a.counts,
                    (const unsigned *)nullptr, (float *)nullptr, (float *)nullptr,
                    (unsigned *)nullptr);
}

hipError_t launch_sort_offsets(hipStream_t st, const SortArgs &a, int grid)
{
    const int nk = a.nr + 1;
    hipError_t e = dispatch_k<true, false>(sort_offsets_kernel, dim3((nk + kOffKeys - 1) / kOffKeys),
                                           dim3(kOffKeys * kOffChunks), 0, st, a.counts, grid, nk,
                                           a.total);
    if (e != hipSuccess) return e;
    return dispatch_k<false, true>(sort_starts_kernel, dim3(1), dim3(1024), 0, st,
                                   (const unsigned *)a.total, nk, a.starts);
}

hipError_t launch_sort_scatter(hipStream_t st, const SortArgs &a, int grid)
{
    return dispatch(a.K > 1 ? sort_pass_kernel<true, true> : sort_pass_kernel<true, false>,
                    dim3(grid), dim3(kPushBlock), sort_lds_bytes(a.nr), st, a.zR, a.zV, a.ids,
                    a.n, a.sub, a.endrot, a.K, a.inv_hr, a.etab, a.fscal, a.nr, a.counts,
                    (const unsigned *)a.starts, a.oR, a.oV, a.oid);
}

hipError_t launch_sort_reduce(hipStream_t st, const SortArgs &a, const float *zR, const float *zV,
                              int n_cu)
{
    (void)n_cu;
    return dispatch(sort_reduce_kernel, dim3(a.nr), dim3(256), 0, st, zR, zV,
                    (const unsigned *)a.starts, (const unsigned *)a.total, a.endrot, a.inv_hr,
                    a.nr, a.hist);
}

hipError_t launch_iota(hipStream_t st, unsigned *ids, int64_t first, int64_t n)
{
    if (n <= 0) return hipSuccess;
    iota_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(ids, first, n);
    return hipGetLastError();
}

hipError_t launch_inverse(hipStream_t st, const unsigned *ids, int64_t n, unsigned *inv)
{
    if (n <= 0) return hipSuccess;
    inverse_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(ids, n, inv);
    return hipGetLastError();
}

hipError_t launch_gather_out(hipStream_t st, const float *zR, const float *zV,
                             const unsigned *inv, int64_t first, int64_t count, double c,
                             double s, double *R, double *V)
{
    if (count <= 0) return hipSuccess;
    gather_out_kernel<<<dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st>>>(
        zR, zV, inv, first, count, c, s, R, V);
    return hipGetLastError();
}

}  // namespace etd
