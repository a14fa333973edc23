// Deterministic sort-by-cell CIC deposit (gfx950).
//
// Per Poisson step, instead of the fused push + LDS-histogram deposit:
//   sort_count_kernel    push each particle in registers (K substeps, frozen
//                        field) and count the cell keys of the new positions
//                        per workgroup (key nr = off the mesh)
//   sort_offsets_kernel  per key, exclusive offsets of the workgroups' counts
//   sort_starts_kernel   exclusive scan of the key totals: segment starts
//   sort_scatter_kernel  push again (same arithmetic, same keys) and write each
//                        particle, with its id, as one 12-byte record to its
//                        slot in cell order.
//                        The particles that workgroup b sends to cell k fill
//                        the contiguous segment (k, b) of the sorted array;
//                        the workgroup sums that segment's CIC weights as it
//                        writes it and stores the sums, one row per workgroup
//   sort_combine_kernel  per node, the sum of the segment sums over the
//                        workgroups in index order
// The weights are the same 2^-32 fixed-point integers as the fused deposit,
// so the node charges are bitwise identical to it; particles within one
// (workgroup, cell) segment may land in any order, which changes no result.
//
// The records: the scatter's stores go to G x N_r slowly filling segments,
// far more open lines than the caches hold, so each store reaches memory as
// a partly filled request of its own; one 12-byte record per particle makes
// one such request where three SoA words made three.  Steps after the first
// of a call read the records (12 B per particle, coalesced), and
// sort_unpack_kernel writes the last step's records back to the SoA state.

#include "pic_device.h"

namespace etd {

namespace {

// LDS of the sort passes, 20 N_r bytes at most (80 KB at N_r = 4096, so two
// workgroups fit a CU): the field table, one slot counter per cell and, in
// the scatter pass, the sum A_k of the node-(k+1) weights of the workgroup's
// particles in cell k (u64).  Off-mesh particles (key N_r) are few: their
// counter is a register (count pass) or the workgroup's global offset entry
// (scatter pass).
struct SortLds {
    float2 *Et;
    unsigned *C;
    unsigned long long *A;
};

__host__ __device__ constexpr size_t sort_sums_offset(int nr)
{
    return ((size_t)nr * sizeof(float2) + (size_t)nr * sizeof(unsigned) + 7) & ~(size_t)7;
}

__device__ __forceinline__ SortLds sort_lds(unsigned char *smem, int nr)
{
    SortLds s;
    s.Et = reinterpret_cast<float2 *>(smem);
    s.C = reinterpret_cast<unsigned *>(smem + (size_t)nr * sizeof(float2));
    s.A = reinterpret_cast<unsigned long long *>(smem + sort_sums_offset(nr));
    return s;
}

// New FP32 state, cell key and CIC weight of one particle after the step.
// FAST: a particle with |z|^2 < lim2 (see on_mesh_limit2) takes the gather
// without range tests; it pays only for several substeps, so the launchers
// choose it for K > 1.
template <bool FAST>
__device__ __forceinline__ void step_one(const MeshView &m, const double4 *__restrict__ sub, int K,
                                         double lim2, double2 er, float &fr, float &fv, int nr,
                                         int &key, double &th)
{
    double zr[1] = {fr}, zv[1] = {fv};
    if (FAST && fma(zr[0], zr[0], zv[0] * zv[0]) < lim2)
        push_group<1, true>(m, sub, K, zr, zv);
    else
        push_group<1>(m, sub, K, zr, zv);
    fr = (float)zr[0];
    fv = (float)zv[0];
    int k;
    key = cell_of(fma(er.x, (double)fr, er.y * (double)fv), m.inv_hr, m.half, m.c, k, th) ? k
                                                                                          : nr;
}

// One particle of the record form: R and V (FP32) and the id, 4-byte aligned,
// so that it is written with one 12-byte store.
struct __attribute__((packed, aligned(4))) SortRec {
    float r, v;
    unsigned id;
};
static_assert(sizeof(SortRec) == 12, "a record is three words");

// Particles 4g .. 4g+3 of a record array: three 16-byte loads, split into
// their R, V and id quadruples.
__device__ __forceinline__ void load_rec_group(const unsigned *__restrict__ rec, int64_t g,
                                               float4 &r4, float4 &v4, uint4 &id4)
{
    const uint4 *q = reinterpret_cast<const uint4 *>(rec) + 3 * g;
    const uint4 a = q[0], b = q[1], c = q[2];
    r4 = make_float4(__uint_as_float(a.x), __uint_as_float(a.w), __uint_as_float(b.z),
                     __uint_as_float(c.y));
    v4 = make_float4(__uint_as_float(a.y), __uint_as_float(b.x), __uint_as_float(b.w),
                     __uint_as_float(c.z));
    id4 = make_uint4(a.z, b.y, c.x, c.w);
}

}  // namespace

// Both passes visit the particles in the same order (groups of four with a
// grid stride, then the ragged tail), so that they assign each particle to
// the same workgroup.  REC: the state before the step is rec_in (records),
// else zR, zV and ids.
template <bool SCATTER, bool FAST, bool REC>
__global__ __launch_bounds__(kPushBlock) void sort_pass_kernel(
    const float *__restrict__ zR, const float *__restrict__ zV, const unsigned *__restrict__ ids,
    const unsigned *__restrict__ rec_in, int64_t n, const double4 *__restrict__ sub,
    const double2 *__restrict__ endrot, int K, double inv_hr, const float2 *__restrict__ etab,
    const double *__restrict__ fscal, int nr, unsigned *__restrict__ counts,
    const unsigned *__restrict__ starts, unsigned *__restrict__ rec_out,
    unsigned long long *__restrict__ sums)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const SortLds L = sort_lds(smem, nr);
    const int tid = threadIdx.x;
    const int nk = nr + 1;
    unsigned *cnt = counts + (size_t)blockIdx.x * nk;
    for (int i = tid; i < nr; i += blockDim.x) {
        L.Et[i] = etab[i];
        L.C[i] = SCATTER ? starts[i] + cnt[i] : 0u;
        if (SCATTER) L.A[i] = 0ull;
    }
    MeshView m;
    m.Et = L.Et;
    m.H = nullptr;
    m.inv_hr = inv_hr;
    m.half = 0.5 * (double)nr;
    m.c = nr >> 1;
    m.Qb = fscal[kQb];
    const double2 er = endrot[0];
    const double lim2 = FAST ? on_mesh_limit2(m, sub, K, fscal[kEmax]) : -1.0;
    const unsigned off_base = SCATTER ? starts[nr] : 0u;
    unsigned n_off = 0u;   // count pass: this thread's off-mesh particles
    __syncthreads();

    SortRec *out = reinterpret_cast<SortRec *>(rec_out);
    auto visit = [&](float fr, float fv, unsigned id) {
        int key;
        double th = 0.0;
        step_one<FAST>(m, sub, K, lim2, er, fr, fv, nr, key, th);
        if (!SCATTER) {
            if (key < nr)
                atomicAdd(&L.C[key], 1u);
            else
                ++n_off;
            return;
        }
        unsigned slot;
        if (key < nr) {
            slot = atomicAdd(&L.C[key], 1u);
            // the particle's weight to node key + 1 goes to its segment's sum
            atomicAdd(&L.A[key], (unsigned long long)fixed_weight(th));
        } else {
            slot = off_base + atomicAdd(&cnt[nr], 1u);
        }
        SortRec o;
        o.r = fr;
        o.v = fv;
        o.id = id;
        out[slot] = o;
    };
    const int64_t n4 = n >> 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + tid; g < n4; g += stride) {
        float4 r4, v4;
        uint4 id4 = make_uint4(0u, 0u, 0u, 0u);
        if (REC) {
            load_rec_group(rec_in, g, r4, v4, id4);
        } else {
            r4 = reinterpret_cast<const float4 *>(zR)[g];
            v4 = reinterpret_cast<const float4 *>(zV)[g];
            if (SCATTER) id4 = reinterpret_cast<const uint4 *>(ids)[g];
        }
        visit(r4.x, v4.x, id4.x);
        visit(r4.y, v4.y, id4.y);
        visit(r4.z, v4.z, id4.z);
        visit(r4.w, v4.w, id4.w);
    }
    const int64_t gt = blockIdx.x * (int64_t)blockDim.x + tid;
    if (gt < n - (n4 << 2)) {
        const int64_t i = (n4 << 2) + gt;
        if (REC) {
            const SortRec q = reinterpret_cast<const SortRec *>(rec_in)[i];
            visit(q.r, q.v, q.id);
        } else {
            visit(zR[i], zV[i], SCATTER ? ids[i] : 0u);
        }
    }
    __syncthreads();
    if (!SCATTER) {
        for (int i = tid; i < nr; i += blockDim.x) cnt[i] = L.C[i];
        // the off-mesh count, summed over the workgroup in the counters'
        // storage, which the loop above has read
        const unsigned wsum = wave_sum(n_off);
        __syncthreads();
        if ((tid & 63) == 0) L.C[tid >> 6] = wsum;
        __syncthreads();
        if (tid == 0) {
            unsigned t = 0u;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += L.C[w];
            cnt[nr] = t;
        }
        return;
    }
    // The workgroup's particles in cell k fill segment (k, b): n_k of them,
    // with node weights sum(2^32 - q) = n_k 2^32 - A_k to node k and A_k to
    // node k + 1.  Row b holds the workgroup's contribution to every node.
    unsigned long long *row = sums + (size_t)blockIdx.x * nk;
    for (int k = tid; k < nk; k += blockDim.x) {
        unsigned long long v = 0ull;
        if (k < nr) {
            const unsigned long long nk_ = (unsigned long long)(L.C[k] - starts[k] - cnt[k]);
            v = (nk_ << 32) - L.A[k];
        }
        if (k > 0) v += L.A[k - 1];
        row[k] = v;
    }
}

// hist[k] = sum over workgroups b = 0 .. G-1 of the segment sums sums[b][k],
// in a fixed order: a workgroup takes 16 nodes; its 16 x 16 threads sum 16
// consecutive chunks of the rows, then one thread per node adds the chunk
// sums in chunk order.
constexpr int kCombKeys = 16, kCombChunks = 16;

__global__ __launch_bounds__(kCombKeys * kCombChunks) void sort_combine_kernel(
    const unsigned long long *__restrict__ sums, int G, int nk,
    unsigned long long *__restrict__ hist)
{
    __shared__ unsigned long long part[kCombChunks][kCombKeys];
    const int kl = threadIdx.x % kCombKeys, ch = threadIdx.x / kCombKeys;
    const int k = blockIdx.x * kCombKeys + kl;
    const int rows = (G + kCombChunks - 1) / kCombChunks;
    const int b0 = ch * rows, b1 = min(b0 + rows, G);
    unsigned long long a = 0ull;
    // integer sums: unrolled, eight loads in flight, the same bits
    if (k < nk)
#pragma unroll 8
        for (int b = b0; b < b1; ++b) a += sums[(size_t)b * nk + k];
    part[ch][kl] = a;
    __syncthreads();
    if (ch == 0 && k < nk) {
        unsigned long long t = 0ull;
        for (int c = 0; c < kCombChunks; ++c) t += part[c][kl];
        hist[k] = t;
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
#pragma unroll 8
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
        int b = b0;
        // eight rows read before any of them is rewritten
        for (; b + 8 <= b1; b += 8) {
            unsigned v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = counts[(size_t)(b + j) * nk + k];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                counts[(size_t)(b + j) * nk + k] = run;
                run += v[j];
            }
        }
        for (; b < b1; ++b) {
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

// The records of one call's last step back to the SoA state (particles 0 ..
// n-1, groups of four with a grid stride, then the ragged tail).
__global__ __launch_bounds__(256) void sort_unpack_kernel(const unsigned *__restrict__ rec,
                                                          int64_t n, float *__restrict__ zR,
                                                          float *__restrict__ zV,
                                                          unsigned *__restrict__ ids)
{
    const int64_t n4 = n >> 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t g = gt; g < n4; g += stride) {
        float4 r4, v4;
        uint4 id4;
        load_rec_group(rec, g, r4, v4, id4);
        reinterpret_cast<float4 *>(zR)[g] = r4;
        reinterpret_cast<float4 *>(zV)[g] = v4;
        reinterpret_cast<uint4 *>(ids)[g] = id4;
    }
    if (gt < n - (n4 << 2)) {
        const int64_t i = (n4 << 2) + gt;
        const SortRec q = reinterpret_cast<const SortRec *>(rec)[i];
        zR[i] = q.r;
        zV[i] = q.v;
        ids[i] = q.id;
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

static size_t sort_lds_bytes(int nr, bool scatter)
{
    return scatter ? sort_sums_offset(nr) + (size_t)nr * sizeof(unsigned long long)
                   : (size_t)nr * sizeof(float2) + (size_t)nr * sizeof(unsigned);
}

size_t sort_lds_bytes_for(int nr) { return sort_lds_bytes(nr, true); }

// The pass kernel for (scatter, K > 1, record input).
typedef void (*SortPassFn)(const float *, const float *, const unsigned *, const unsigned *,
                           int64_t, const double4 *, const double2 *, int, double, const float2 *,
                           const double *, int, unsigned *, const unsigned *, unsigned *,
                           unsigned long long *);

static SortPassFn sort_pass_fn(bool scatter, bool fast, bool rec)
{
    static const SortPassFn tab[8] = {
        sort_pass_kernel<false, false, false>, sort_pass_kernel<false, false, true>,
        sort_pass_kernel<false, true, false>,  sort_pass_kernel<false, true, true>,
        sort_pass_kernel<true, false, false>,  sort_pass_kernel<true, false, true>,
        sort_pass_kernel<true, true, false>,   sort_pass_kernel<true, true, true>};
    return tab[(scatter ? 4 : 0) + (fast ? 2 : 0) + (rec ? 1 : 0)];
}

hipError_t setup_sort_lds(int nr)
{
    hipError_t e;
    for (int v = 0; v < 8; ++v) {
        const bool scatter = v >= 4;
        const void *f = reinterpret_cast<const void *>(sort_pass_fn(scatter, v & 2, v & 1));
        if ((e = raise_dynamic_lds(f, (int)sort_lds_bytes(nr, scatter))) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_sort_count(hipStream_t st, const SortArgs &a, int grid)
{
    return dispatch(sort_pass_fn(false, a.K > 1, a.rec_in != nullptr), dim3(grid),
                    dim3(kPushBlock), sort_lds_bytes(a.nr, false), st, a.zR, a.zV, a.ids,
                    a.rec_in, a.n, a.sub, a.endrot, a.K, a.inv_hr, a.etab, a.fscal, a.nr,
                    a.counts, (const unsigned *)nullptr, (unsigned *)nullptr,
                    (unsigned long long *)nullptr);
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
    return dispatch(sort_pass_fn(true, a.K > 1, a.rec_in != nullptr), dim3(grid),
                    dim3(kPushBlock), sort_lds_bytes(a.nr, true), st, a.zR, a.zV, a.ids,
                    a.rec_in, a.n, a.sub, a.endrot, a.K, a.inv_hr, a.etab, a.fscal, a.nr,
                    a.counts, (const unsigned *)a.starts, a.rec_out, a.sums);
}

hipError_t launch_sort_unpack(hipStream_t st, const unsigned *rec, int64_t n, float *zR, float *zV,
                              unsigned *ids)
{
    if (n <= 0) return hipSuccess;
    int64_t g = ((n >> 2) + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return dispatch(sort_unpack_kernel, dim3((unsigned)g), dim3(256), 0, st, rec, n, zR, zV, ids);
}

hipError_t launch_sort_combine(hipStream_t st, const SortArgs &a, int grid)
{
    const int nk = a.nr + 1;
    return dispatch(sort_combine_kernel, dim3((nk + kCombKeys - 1) / kCombKeys),
                    dim3(kCombKeys * kCombChunks), 0, st, (const unsigned long long *)a.sums, grid,
                    nk, a.hist);
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
