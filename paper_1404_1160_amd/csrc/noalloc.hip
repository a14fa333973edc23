// The plain step for callers that cannot allocate device memory
// (ep_step_noalloc): code under HIP graph capture, serving loops, harnesses
// that forbid allocation.  The caller passes its FP32 rotating-frame particle
// arrays; every other buffer the step's kernels use -- the fixed-point charge
// histogram, the FP32 gather table, the FP64 node arrays, the field scalars and
// the substep coefficient tables -- lives in one static device array of
// modest, fixed size, which each device the library runs on holds until the
// process ends.  The kernels are those of ep_step, launched in the same order
// with the same arguments, so the results are ep_step's.

#include <mutex>

#include "context.h"

using namespace etd;

namespace {

constexpr int kMaxDevices = 64;
// Substep coefficients per table fill: the step tables are filled in pieces of
// at most kStaticEntries / K steps.
constexpr size_t kStaticEntries = size_t(1) << 15;

constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

constexpr size_t kNodes = (size_t)kMaxCells + 1;
constexpr size_t kOffHist = 0;                                           // u64 [nr + 1]
constexpr size_t kOffEtab = kOffHist + align256(kNodes * 8);             // float2 [nr]
constexpr size_t kOffRho = kOffEtab + align256((size_t)kMaxCells * 8);   // double [nr + 1]
constexpr size_t kOffE = kOffRho + align256(kNodes * 8);                 // double [nr + 1]
constexpr size_t kOffFscal = kOffE + align256(kNodes * 8);               // double [kFieldScalars]
constexpr size_t kOffSub = kOffFscal + 256;                              // double4 [kStaticEntries]
constexpr size_t kOffEndrot = kOffSub + kStaticEntries * sizeof(double4);  // double2 [...]
constexpr size_t kScratchBytes = kOffEndrot + kStaticEntries * sizeof(double2);

static_assert(kFieldScalars * sizeof(double) <= 256, "field scalars fit their slot");

}  // namespace

// The step's working memory on each device (about 1.8 MB).  In host code this
// name stands for the host-side shadow of the variable, not for device memory:
// the device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
unsigned char *g_scratch[kMaxDevices];   // device address of `scratch` on each device
int g_n_cu[kMaxDevices];

// Once per device, with that device current: the address of its copy of
// `scratch` and its compute-unit count.
hipError_t device_slot(int dev, unsigned char **ptr, int *n_cu)
{
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        unsigned char *p = nullptr;
        hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        int cu = 0;
        e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        g_n_cu[dev] = cu;
        g_scratch[dev] = p;
    }
    *ptr = g_scratch[dev];
    *n_cu = g_n_cu[dev];
    return hipSuccess;
}

__global__ void clear_u64_kernel(unsigned long long *__restrict__ x, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0ull;
}

ep_status fail(ep_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    set_context_free_error(buf);
    return code;
}

ep_status hipfail(const char *what, hipError_t e)
{
    return fail(EP_EHIP, "ep_step_noalloc: %s: %s", what, hipGetErrorString(e));
}

#define NA_CHK(expr)                                \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return hipfail(#expr, e_); \
    } while (0)

}  // namespace

extern "C" ep_status ep_step_noalloc(float *zR, float *zV, uint64_t n, double w,
                                     uint32_t n_cells, double r_max, uint32_t substeps,
                                     double dt, double eps, int32_t field, uint64_t n_steps,
                                     double *phase, int32_t device, void *hip_stream)
{
    if (!phase || !isfinite(*phase) || !(dt > 0.0) || !(eps > 0.0) || !isfinite(dt) ||
        !isfinite(eps) ||
        (field != EP_FIELD_ZERO && field != EP_FIELD_DUFFING && field != EP_FIELD_POISSON))
        return fail(EP_EINVAL, "ep_step_noalloc: need a finite phase, dt > 0, eps > 0 and a "
                               "valid field model");
    if (n > kMaxParticles || !(w > 0.0) || !isfinite(w) ||
        (n > 0 && (!zR || !zV || (reinterpret_cast<uintptr_t>(zR) & 15) ||
                   (reinterpret_cast<uintptr_t>(zV) & 15))))
        return fail(EP_EINVAL, "ep_step_noalloc: need n < 2^31 particles in 16-byte aligned "
                               "device arrays and a weight w > 0");
    if (substeps == 0 || substeps > kStaticEntries)
        return fail(EP_EINVAL, "ep_step_noalloc: substeps %u outside 1..%zu (the static "
                               "coefficient table holds %zu entries)",
                    substeps, kStaticEntries, kStaticEntries);
    if (field == EP_FIELD_POISSON &&
        (n_cells < 2 || (n_cells & 1) || n_cells > kMaxCells || !(r_max > 0.0) ||
         !isfinite(r_max)))
        return fail(EP_EINVAL, "ep_step_noalloc: need an even mesh of 2..%u cells (the static "
                               "mesh buffers' size) and r_max > 0",
                    kMaxCells);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev ||
        device >= kMaxDevices)
        return fail(EP_EINVAL, "ep_step_noalloc: no such HIP device");
    if (n_steps == 0) return EP_OK;
    const int K = (int)substeps;
    const double dphi = fmod(dt / eps, kTwoPi);
    if (field == EP_FIELD_ZERO) {
        // E = 0: the rotating-frame state is unchanged; only the phase advances
        *phase = fmod(*phase + (double)n_steps * dphi, kTwoPi);
        return EP_OK;
    }
    DeviceGuard guard(device);
    unsigned char *base = nullptr;
    int n_cu = 0;
    NA_CHK(device_slot(device, &base, &n_cu));
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const double theta = dt / ((double)K * eps);
    const double h = dt / (double)K;
    StepTables tab;
    tab.sub = reinterpret_cast<double4 *>(base + kOffSub);
    tab.endrot = reinterpret_cast<double2 *>(base + kOffEndrot);
    MeshArgs ma{};
    const int grid_cap = n_cu * 16;
    if (field == EP_FIELD_POISSON) {
        const int nr = (int)n_cells;
        ma.nr = nr;
        ma.w = w;
        ma.hr = 2.0 * r_max / (double)nr;
        ma.hist = reinterpret_cast<unsigned long long *>(base + kOffHist);
        ma.etab = reinterpret_cast<float2 *>(base + kOffEtab);
        ma.rho64 = reinterpret_cast<double *>(base + kOffRho);
        ma.E64 = reinterpret_cast<double *>(base + kOffE);
        ma.Psi64 = nullptr;   // the field-only solve writes no potential
        ma.fscal = reinterpret_cast<double *>(base + kOffFscal);
        NA_CHK(setup_mesh_lds(nr));
        // the histogram starts at zero (a fill kernel: callers may capture
        // this call into a graph); each solve clears it again after reading
        clear_u64_kernel<<<dim3((nr + 1 + 255) / 256), dim3(256), 0, st>>>(ma.hist, nr + 1);
        NA_CHK(hipGetLastError());
        // field of the current state, as the context path computes it
        const double2 er = make_double2(cos(*phase), sin(*phase));
        NA_CHK(launch_push_poisson(st, false, zR, zV, (int64_t)n, nullptr, nullptr, er, 0, ma,
                                   grid_cap));
        NA_CHK(launch_mesh_solve(st, ma, false));
    }
    // steps are grouped as ep_step groups them (the same phase bookkeeping);
    // each group's coefficients are made in pieces that fit the static table
    size_t chunk = kTableEntries / (size_t)K;
    if (chunk < 1) chunk = 1;
    const int64_t piece = (int64_t)(kStaticEntries / (size_t)K);
    double p = *phase;
    uint64_t done = 0;
    while (done < n_steps) {
        const uint64_t rem = n_steps - done;
        const int S = (int)(rem < chunk ? rem : chunk);
        for (int64_t j0 = 0; j0 < S; j0 += piece) {
            const int s = (int)(S - j0 < piece ? S - j0 : piece);
            NA_CHK(launch_phase_table(st, tab, p, dphi, theta, h, K, s, j0));
            if (field == EP_FIELD_DUFFING) {
                NA_CHK(launch_push_duffing(st, zR, zV, (int64_t)n, tab.sub, K, s));
                continue;
            }
            for (int j = 0; j < s; ++j) {
                NA_CHK(launch_push_poisson(st, true, zR, zV, (int64_t)n, tab.sub + (size_t)j * K,
                                           tab.endrot + j, make_double2(1.0, 0.0), K, ma,
                                           grid_cap));
                NA_CHK(launch_mesh_solve(st, ma, false));
            }
        }
        p = fmod(p + (double)S * dphi, kTwoPi);
        done += (uint64_t)S;
    }
    *phase = p;
    return EP_OK;
}
