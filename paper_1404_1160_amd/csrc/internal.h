// Internal launcher declarations shared by the kernels and the host runtime.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace etd {

// Kernel timing: events that the next dispatch of this host thread carries.
// hipExtLaunchKernel attaches them to the dispatch packet itself, so a timed
// run adds no marker packets (and no gaps) between kernels.  `start` goes to
// the first kernel of a timed launcher and `stop` to its last.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
LaunchEvents &next_launch_events();

// Launch `kernel`, consuming the pending start event (FIRST) and/or stop
// event (LAST); with no events pending this is a plain launch.
template <bool FIRST, bool LAST, typename F, typename... Args>
inline hipError_t dispatch_k(F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                             Args... args)
{
    LaunchEvents &ev = next_launch_events();
    hipEvent_t a = nullptr, b = nullptr;
    if (FIRST) {
        a = ev.start;
        ev.start = nullptr;
    }
    if (LAST) {
        b = ev.stop;
        ev.stop = nullptr;
    }
    hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)lds, st, a, b, 0u, args...);
    return hipGetLastError();
}

template <typename F, typename... Args>
inline hipError_t dispatch(F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                           Args... args)
{
    return dispatch_k<true, true>(kernel, grid, block, lds, st, args...);
}

// Raise a kernel's dynamic-LDS limit to at least `bytes`.  The limit is a
// property of the kernel in the process, shared by every context: it only ever
// grows, so a context with a smaller mesh cannot lower it under another's.
hipError_t raise_dynamic_lds(const void *kernel, int bytes);

constexpr int kPushBlock = 1024;       // threads per block of the mesh push kernels
constexpr int kSolveBlock = 1024;      // threads of the single-block mesh solve
constexpr int kMomentBlock = 256;
constexpr int kMomentQuantities = 4;   // sum R^2, sum |z|^2, sum R^4, (unused)
constexpr int kMomentCounts = 2;       // off-mesh, non-finite

// Scalars of the solved field, stored on the device after each solve.
// kEmax: an upper bound on |E| of the CIC gather anywhere on the mesh
enum FieldScalar { kQb = 0, kFieldEnergy = 1, kMeshCharge = 2, kEmax = 3, kFieldScalars = 4 };

// Per-substep coefficients of the plain push (FP64): the midpoint phase phi
// of the substep gives (cos phi, sin phi, h sin phi, h cos phi).
struct StepTables {
    double4 *sub;     // [S*K]
    double2 *endrot;  // [S]  (cos, sin) of the phase at the end of each step
};

hipError_t launch_phase_table(hipStream_t st, StepTables tab, double phi0, double dphi,
                              double theta, double h, int K, int S, int64_t j0 = 0);

hipError_t launch_twist_in(hipStream_t st, const double *R, const double *V, float *zR,
                           float *zV, int64_t n, double c, double s);
hipError_t launch_twist_out(hipStream_t st, const float *zR, const float *zV, double *R,
                            double *V, int64_t n, double c, double s);

hipError_t launch_push_duffing(hipStream_t st, float *zR, float *zV, int64_t n,
                               const double4 *sub, int K, int S);

// Device arrays and scalars of the mesh.
struct MeshArgs {
    int nr;                   // cells
    double w;                 // particle weight
    double hr;                // cell width
    unsigned long long *hist; // [nr+1] fixed-point node charges being accumulated
    float2 *etab;             // [nr]   FP32 gather table (E_m, E_{m+1} - E_m)
    double *rho64, *E64, *Psi64;  // [nr+1] FP64 node values
    double *fscal;            // [kFieldScalars]
};

// One Poisson step: K-substep push in the frozen field, then CIC deposit of
// the new positions into hist (fixed point, 2^-32 of a particle weight).  The
// rotation to the lab frame at the end of the step is endrot_tab[0] if
// endrot_tab is non-null, else endrot_val.  With push == false only the
// deposit of the current state is done.
hipError_t launch_push_poisson(hipStream_t st, bool push, float *zR, float *zV, int64_t n,
                               const double4 *sub, const double2 *endrot_tab, double2 endrot_val,
                               int K, const MeshArgs &ma, int grid_cap);

// Raise the dynamic LDS limit of the mesh kernels for an nr-cell mesh.
hipError_t setup_mesh_lds(int nr);
size_t push_lds_bytes_for(int nr);

// Field of the accumulated charge; with potential also Psi and the field
// energy (else they are left as they were).
hipError_t launch_mesh_solve(hipStream_t st, const MeshArgs &ma, bool potential);
// Psi and the field energy of the field in E64 (the same bits as a solve
// with potential).
hipError_t launch_potential(hipStream_t st, const MeshArgs &ma);

// ------------------------------------------------------------ sorted deposit

// Inside one multi-step call the sorted state travels as 12-byte records
// (R, V as FP32 bits, id), so that the scatter stores one record per particle
// instead of three scattered words; the first step of a call reads the SoA
// state, and sort_unpack writes the last step's records back to it.
struct SortArgs {
    const float *zR, *zV;      // state before the step (particle order), if rec_in is null
    const unsigned *ids;       // particle ids in that order, if rec_in is null
    const unsigned *rec_in;    // or the state as records [n][3]
    int64_t n;
    const double4 *sub;        // substep table of the step
    const double2 *endrot;     // rotation to the lab frame at the end of the step
    int K;
    double inv_hr;
    const float2 *etab;        // frozen field
    const double *fscal;
    int nr;
    unsigned *counts;          // [grid][nr+1]
    unsigned *total;           // [nr+1]
    unsigned *starts;          // [nr+1]
    unsigned *rec_out;         // state after the step, cell order, records [n][3]
    unsigned long long *hist;  // [nr+1] fixed-point node charges
    unsigned long long *sums;  // [grid][nr+1] segment sums of the scatter pass
};

hipError_t setup_sort_lds(int nr);
hipError_t launch_sort_count(hipStream_t st, const SortArgs &a, int grid);
hipError_t launch_sort_offsets(hipStream_t st, const SortArgs &a, int grid);
hipError_t launch_sort_scatter(hipStream_t st, const SortArgs &a, int grid);
hipError_t launch_sort_combine(hipStream_t st, const SortArgs &a, int grid);
hipError_t launch_sort_unpack(hipStream_t st, const unsigned *rec, int64_t n, float *zR, float *zV,
                              unsigned *ids);
size_t sort_lds_bytes_for(int nr);   // LDS of the scatter pass (the larger one)
hipError_t launch_iota(hipStream_t st, unsigned *ids, int64_t first, int64_t n);
hipError_t launch_inverse(hipStream_t st, const unsigned *ids, int64_t n, unsigned *inv);
hipError_t launch_gather_f32(hipStream_t st, const float *zR, const float *zV, const unsigned *inv,
                             int64_t n, float *oR, float *oV);
hipError_t launch_gather_out(hipStream_t st, const float *zR, const float *zV,
                             const unsigned *inv, int64_t first, int64_t count, double c,
                             double s, double *R, double *V);

// ------------------------------------------------------------ learned corrector

constexpr int kH = 64;    // hidden width
constexpr int kOut = 2;   // outputs (delta, kappa)

__host__ __device__ constexpr int mlp_n_params(int n_in)
{
    return kH * n_in + kH + kH * kH + kH + kOut * kH + kOut;
}

// Inference constants of a trained network for one (dt, eps).
struct MlpInfer {
    // FP16 MFMA A-fragments (uint4 = 8 FP16 values of one lane).  Hidden unit
    // order in k: step kk, lane group g, element e stands for unit
    //   32 (kk / 2) + 16 (kk % 2) + 8 (e / 4) + 4 g + e % 4,
    // the unit whose result lane (., g) holds in accumulator element
    // 8 (kk % 2) + e of tile kk / 2.
    // FP16 (fp16 != 0) or BF16 values; with BF16 the W2 and W3 fragments
    // are followed by those of their lo parts (w - hi).
    const uint4 *w1f;    // [2 tiles][64 lanes] layer 1 / 64, features folded (see kernel)
    const uint4 *w2f;    // [(2)][8 = 4 mt + kk][64 lanes] W2 / 64
    const float4 *b2;    // [16] b2 / 64
    const uint4 *w3f;    // [(2)][4 kk][64 lanes] W3, rows 0, 1 the outputs, the rest zero
    float b3_0, b3_1, mu_d, sig_d, mu_k, sig_k;
    float xmax;          // features are clamped to +-xmax
    int fp16;            // MFMA operands in FP16 (1) or BF16 (0)
    int scaled;          // outputs are (a delta, a kappa), a = |y|, instead of (delta, kappa)
    int project;         // particles that pass are projected radially onto their energy shell
};

// Labels (delta, kappa), or (a delta, a kappa) with scaled != 0, around the
// free rotation (Kb = 0) or the plain push with Kb substeps (table bsub).
hipError_t launch_gen_labels_duffing(hipStream_t st, const float *R, const float *V, int64_t n,
                                     const double4 *sub, int K, const double4 *bsub, int Kb,
                                     float inv_sin, float c_phi, float s_phi, float th_scaled,
                                     int scaled, float *X, float *Y);
// Plain Kb-substep Duffing push of every particle from z into c (FP32).
hipError_t launch_base_push_duffing(hipStream_t st, const float *zR, const float *zV, float *cR,
                                    float *cV, int64_t n, const double4 *sub, int Kb);
hipError_t setup_train_lds(int n_in);
// Gradient of the MSE loss over samples [first, first + batch) (X: [.][n_in],
// Y: [.][2] raw labels, norm = {mu_d, 1/sig_d, mu_k, 1/sig_k}).
hipError_t launch_mlp_grad(hipStream_t st, int n_in, const float *params, const float *X,
                           const float *Y, int64_t first, int batch, const float norm[4],
                           float *gpart, float *lpart, float *grad, float *loss);
// One Adam step on the batch whose sample s is row first + s * sstride.
hipError_t launch_mlp_train_step(hipStream_t st, int n_in, float *params, float *m, float *v,
                                 const float *X, const float *Y, int64_t first, int64_t sstride,
                                 int batch, const float norm[4], float *gpart, float *lpart,
                                 float *grad, float *loss, float lr, float b1, float b2, float bc1,
                                 float bc2, float eps);
// Learned Duffing step: network prediction, energy check |dH| <= tol |H|,
// passing particles updated in place, failing ones appended to queue.  The
// polar map acts around z (cR == nullptr) or around the base push's c.
hipError_t launch_mlp_push_duffing(hipStream_t st, float *zR, float *zV, const float *cR,
                                   const float *cV, int64_t n, const MlpInfer &net, double2 rot0,
                                   double2 rot1, double eps, double tol, unsigned *qcount,
                                   unsigned *queue, int n_cu);
// Energy projection of the fallback particles (as for the network's, with an
// FP64 Newton step): on/off, the step's start and end phases, 1/(2 eps).
struct FallbackProjection {
    int on;
    double2 rot0, rot1;
    double inv2eps;
};
// Plain K-substep Duffing push of the *qcount queued particles; adds the count
// to *total.
hipError_t launch_fallback_duffing(hipStream_t st, float *zR, float *zV, const unsigned *queue,
                                   const unsigned *qcount, const double4 *sub, int K,
                                   const FallbackProjection &proj, unsigned long long *total,
                                   int n_cu);
hipError_t launch_gen_labels_poisson(hipStream_t st, const float *zR, const float *zV,
                                     int64_t first, int64_t stride, int64_t count, double2 rot0,
                                     const MeshArgs &ma, const double4 *sub, int K, float inv_sin,
                                     float c_phi, float s_phi, float th_scaled, float inv_sE,
                                     int scaled, float *X, float *Y);
// Learned step in the frozen Poisson field: 6-input network, energy check
// with the mesh potential, CIC deposit of the particles that pass.
hipError_t launch_mlp_push_poisson(hipStream_t st, float *zR, float *zV, int64_t n,
                                   const MlpInfer &net, double2 rot0, double2 rot1, double eps,
                                   double tol, unsigned *qcount, unsigned *queue,
                                   const MeshArgs &ma, double rmax, int n_cu);
// Plain push + deposit of the queued particles in the frozen Poisson field
// (er: end-of-step phase; proj.rot1 is er).
hipError_t launch_fallback_poisson(hipStream_t st, float *zR, float *zV, const unsigned *queue,
                                   const unsigned *qcount, const double4 *sub, int K, double2 er,
                                   const MeshArgs &ma, double rmax, const FallbackProjection &proj,
                                   unsigned long long *total, int n_cu);
hipError_t setup_learned_lds(int nr);

// ------------------------------------------------------------ fine solvers
// Per-particle FP64 state of the lock-step fine solves (Poisson field).
struct FineArgs {
    double *yR, *yV;            // current fine level
    double *sR, *sV;            // RK4 stage state
    double *aR, *aV;            // RK4 accumulator k1 + 2 k2 + 2 k3
    double *pR, *pV;            // level L-2 (captures)
    double *cR, *cV, *dR, *dV;  // captured y(t_n + o) and y(t_n + o + T)
    double *t1, *T, *o;         // first sign change, period, remainder
    int *cnt;                   // sign changes found
    long long *N;               // whole periods
    unsigned long long *done, *last, *unresolved;  // [1] each
    double *red;                // 257: partial sums of a fixed-order reduction, result
};
hipError_t launch_rk4_duffing(hipStream_t st, float *zR, float *zV, int64_t n, double h,
                              double eps, long long steps, double2 rot0, double2 rot1);
// reuse: T already holds the periods and the search is skipped
hipError_t launch_ietd_duffing(hipStream_t st, float *zR, float *zV, int64_t n, double dt,
                               double h, double eps, long long max_fine, double2 rot0,
                               double2 rot1, bool reuse, double *T, long long *N,
                               unsigned long long *unresolved);
// stage 1-4 of the coupled RK4 step to level L; mode 0 reference, 1 period
// search, 2 captures
hipError_t launch_rk4_stage(hipStream_t st, int stage, int mode, const FineArgs &a, int64_t n,
                            double h, double eps, long long L, const MeshArgs &ma, int grid_cap);
hipError_t launch_fine_deposit(hipStream_t st, const double *yR, int64_t n, const MeshArgs &ma,
                               int grid_cap);
hipError_t launch_fine_begin(hipStream_t st, const FineArgs &a, const float *zR, const float *zV,
                             int64_t n, double2 rot0, int mode, double eps);
hipError_t launch_ietd_split(hipStream_t st, const FineArgs &a, int64_t n, double dt, double h);
hipError_t launch_fine_end(hipStream_t st, const FineArgs &a, float *zR, float *zV, int64_t n,
                           double2 rot1, int ietd);
hipError_t setup_fine_lds(int nr);
hipError_t launch_period_duffing(hipStream_t st, const float *zR, const float *zV, int64_t n,
                                 double h, double eps, long long max_fine, double2 rot0, double *T,
                                 unsigned long long *unresolved);
hipError_t launch_cetd_duffing(hipStream_t st, float *zR, float *zV, int64_t n, double hP,
                               long long K1, double ho, long long K2, double q, double eps,
                               double2 rot0, double2 rot1);
// fixed-order sum of x[0..n) into *out (partial: g doubles)
hipError_t launch_sum(hipStream_t st, const double *x, int64_t n, double *partial, int g,
                      double *out);
hipError_t launch_fill_ll(hipStream_t st, long long *x, int64_t n, long long v);
hipError_t launch_cetd_combine(hipStream_t st, const FineArgs &a, int64_t n, double q);

hipError_t launch_moments(hipStream_t st, const float *zR, const float *zV, int64_t n,
                          double c, double s, double rmax, double *partial,
                          unsigned long long *pcount, int grid, double *out,
                          unsigned long long *out_count);

int moments_grid(int64_t n);

}  // namespace etd
