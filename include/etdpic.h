/*
 * etdpic.h: C ABI of the exponential-integrator Particle-In-Cell step on
 * AMD Instinct MI355X (gfx950).
 *
 * The library advances a beam of macroparticles (R_i, V_i) with uniform weight
 * w along the stiff characteristics of the axisymmetric-beam Vlasov equation
 *     dR/dt = V/eps,  dV/dt = -R/eps + E(R, t)
 * (Frenod, Hirstoaga, Lutz, arXiv 1404.1160: eq. 1.1 and its characteristics
 * eq. 1.4).  The eps-linear part is integrated exactly by the rotation r of
 * eq. 3.3 (T = 2 pi), and E enters through the variation-of-constants
 * (Duhamel) integral of eq. 3.6, evaluated by the midpoint rule along the free
 * rotation on K substeps per macro step.  E is either the given field
 * E = -R^3 (eq. 1.3) or the self-consistent field of the Poisson equation
 * d/dr (r E) = rho (eq. 1.2), obtained by a cloud-in-cell (CIC) deposit of the
 * charge onto a radial mesh, a trapezoidal prefix sum over the cells
 * (section 2.3) and a CIC gather back to the particles.
 *
 * Conventions for every entry point:
 *   - Every function returns an ep_status: EP_OK (0) or a negative code; no
 *     exception or signal crosses the ABI.  ep_last_error() gives the message.
 *   - Host arrays are owned by the caller and only read or written during the
 *     call; device memory is owned by the library unless bound with
 *     ep_bind_particles().
 *   - Work is queued on the context's HIP stream; ep_step() returns before the
 *     GPU finishes.  Calls that return host data synchronise that stream and
 *     report asynchronous HIP errors as EP_EHIP.
 *   - One context may be used by one host thread at a time.
 */
#ifndef ETDPIC_H
#define ETDPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ep_ctx ep_ctx;

typedef enum {
    EP_OK = 0,
    EP_EINVAL = -1,      /* an argument is out of range or inconsistent        */
    EP_ENOMEM = -2,      /* device or host allocation failed                   */
    EP_EHIP = -3,        /* a HIP call or a kernel failed                      */
    EP_ESTATE = -4,      /* the call does not fit the context's state          */
    EP_ENOTRAINED = -5,  /* learned push requested with no network loaded      */
    EP_EIO = -6          /* checkpoint file could not be read or written       */
} ep_status;

typedef enum {
    EP_FIELD_ZERO = 0,     /* E = 0: free rotation with period 2 pi eps (section 1) */
    EP_FIELD_DUFFING = 1,  /* E = -R^3 (eq. 1.3)                                    */
    EP_FIELD_POISSON = 2   /* d/dr (r E) = rho (eq. 1.2) on the radial mesh         */
} ep_field;

typedef enum {
    EP_DEPOSIT_ATOMIC = 0, /* per-workgroup LDS histograms in 2^-32 fixed point      */
    EP_DEPOSIT_SORTED = 1  /* particles reordered by cell, segmented reduction       */
} ep_deposit;

typedef enum {
    EP_PUSH_PLAIN = 0,     /* K-substep midpoint quadrature of the Duhamel term      */
    EP_PUSH_LEARNED = 1,   /* MLP prediction of the Duhamel term, energy-checked,
                              with the plain push as fallback                         */
    EP_PUSH_RK4 = 2,       /* the paper's reference: classic RK4 on eq. 1.4 with a
                              small step, field re-solved at every stage             */
    EP_PUSH_IMPROVED_ETD = 3, /* the paper's improved ETD scheme (Algorithm 3.4)     */
    EP_PUSH_CLASSIC_ETD = 4,  /* Algorithm 2.1 with the fast period 2 pi eps          */
    EP_PUSH_MODIFIED_ETD = 5  /* Algorithm 2.1 with the mean of the particles' periods */
} ep_push;

/* Context configuration (ep_create).
 *   n_particles : capacity of the particle arrays (1 <= n_particles < 2^31).
 *   n_cells     : N_r, number of mesh cells; even, 2 <= N_r <= 8192.  The mesh
 *                 has N_r + 1 nodes x_k = -r_max + k h_r, h_r = 2 r_max / N_r,
 *                 with the centre node x_{N_r/2} = 0.
 *   substeps    : K >= 1, substeps per macro step of the plain push.
 *   r_max       : half width of the mesh, > 0.
 *   deposit     : ep_deposit.
 *   device      : HIP device ordinal.
 *   hip_stream  : hipStream_t to queue work on, or NULL for a library-owned
 *                 stream (created at default priority).  A caller's stream
 *                 (and bound arrays, ep_bind_particles) must come from the
 *                 same HIP runtime the library is linked with: a framework
 *                 that ships its own copy of the runtime cannot share them. */
typedef struct {
    uint64_t n_particles;
    uint32_t n_cells;
    uint32_t substeps;
    double r_max;
    int32_t deposit;
    int32_t device;
    void *hip_stream;
} ep_config;

/* Diagnostics of the current time level (ep_moments).  Sums are over all
 * particles with weight w, accumulated in FP64 in a fixed order.
 *   t, phase        : simulated time and the accumulated fast phase t/eps
 *                     reduced mod 2 pi (both FP64)
 *   charge          : w * N
 *   rms_radius      : sqrt(sum w R^2 / charge)   (NaN particles excluded)
 *   kinetic         : sum w (R^2 + V^2) / (2 eps)
 *   potential       : Duffing: sum w R^4 / 4;  Poisson: int_0^{r_max} x E(x)^2 dx
 *                     (trapezoid on the nodes of the current field); 0 for E = 0
 *   energy          : kinetic + potential
 *   n_offmesh       : particles with R outside [-r_max, r_max)
 *   n_nan           : particles whose R or V is not finite
 *   n_fallback      : particles that took the plain push in the last learned step */
typedef struct {
    double t;
    double phase;
    double charge;
    double rms_radius;
    double energy;
    double kinetic;
    double potential;
    uint64_t n_steps;
    uint64_t n_offmesh;
    uint64_t n_nan;
    uint64_t n_fallback;
} ep_moments;

/* Create a context on cfg->device and allocate its device buffers.
 * n_particles must be below 2^31: the exact-integer trapezoid scan of the
 * charge sums up to 2 N 2^32 in 64 bits, and the learned push's fallback
 * queue holds 32-bit particle indices.
 * Errors: EP_EINVAL (bad sizes), EP_ENOMEM, EP_EHIP. */
ep_status ep_create(const ep_config *cfg, ep_ctx **out);

/* Release the context and all device memory it owns.  NULL is accepted. */
ep_status ep_destroy(ep_ctx *ctx);

/* Message of the last failed call on ctx (or, when ctx is NULL, of the last
 * failed call without a context: ep_create, ep_step_noalloc).  Valid until the
 * next call on the same context. */
const char *ep_last_error(const ep_ctx *ctx);

/* Load n <= capacity particles (host FP64 arrays R[n], V[n], lab frame) with
 * uniform weight w > 0 as the state at the current time level.  The library
 * stores them in FP32 in the frame rotating with the free flow,
 * z = r(-t/eps) y (eq. 3.3), so that the exact rotation is never applied to the
 * stored state.  Invalidates the mesh field.  Errors: EP_EINVAL, EP_EHIP. */
ep_status ep_set_particles(ep_ctx *ctx, const double *R, const double *V, uint64_t n,
                           double w);

/* Use caller-owned device arrays zR_dev[n], zV_dev[n] (FP32, rotating frame at
 * the current time level, 16-byte aligned) as the particle state instead of the
 * library's own.  The caller keeps them alive until ep_destroy or the next
 * bind.  n <= capacity.  Errors: EP_EINVAL. */
ep_status ep_bind_particles(ep_ctx *ctx, float *zR_dev, float *zV_dev, uint64_t n, double w);

/* Advance n_steps macro steps of size dt > 0 at parameter eps > 0 in the field
 * model `field` (ep_field).  Each step: exact rotation by dt/eps, Duhamel term
 * by K-substep midpoint quadrature with E frozen at t_n (Poisson: deposit,
 * prefix-sum solve and gather, section 2.3), or the learned push when enabled.
 * dt and eps may change between calls; the phase t/eps is carried in FP64.
 * With EP_DEPOSIT_SORTED each Poisson step leaves the particles in cell order
 * (ep_get_particles and checkpoints still use the loaded order); between the
 * steps of one call the state is kept as 12-byte (R, V, id) records, and the
 * call ends with one pass that writes them back to the FP32 state, so a call
 * of n steps costs n sorted steps and one such pass.
 * Asynchronous.  Errors: EP_EINVAL, EP_ESTATE (no particles), EP_EHIP. */
ep_status ep_step(ep_ctx *ctx, double dt, double eps, int32_t field, uint64_t n_steps);

/* Moments of the current state (see ep_moments), with eps and field naming the
 * energy to report.  Synchronises.  Errors: EP_EINVAL, EP_ESTATE, EP_EHIP. */
ep_status ep_moments_get(ep_ctx *ctx, double eps, int32_t field, ep_moments *out);

/* Copy particles [offset, offset + count) of the current state to host FP64
 * arrays R[count], V[count] (lab frame: the FP32 rotating-frame values are
 * rotated back in FP64).  offset + count must not exceed the loaded count.
 * Synchronises.  Errors: EP_EINVAL, EP_EHIP. */
ep_status ep_get_particles(ep_ctx *ctx, double *R, double *V, uint64_t offset, uint64_t count);

/* Mesh field of the current particle positions (deposited and solved first if
 * stale): rho, E and the potential Psi (Psi(0) = 0, -Psi' = E) at the
 * n_nodes = N_r + 1 nodes, FP64, and the half enclosed charge Qb at the mesh
 * edge (off the mesh E = Qb / R).  Any output pointer may be NULL.
 * Synchronises.  Errors: EP_EINVAL, EP_ESTATE, EP_EHIP. */
ep_status ep_get_field(ep_ctx *ctx, double *rho, double *E, double *Psi, double *Qb,
                       uint32_t n_nodes);

/* Select the push (ep_push).  For EP_PUSH_LEARNED: drift_tol is the per-particle
 * relative energy-drift bound |H(y_{n+1}) - H(y_n)| <= drift_tol * H(y_n)
 * (H(y) = |y|^2/(2 eps) + P(R), the frozen-field energy of the step: P = R^4/4
 * for the Duffing field, the mesh potential Psi^n for the Poisson field), and
 * fallback_substeps the K used by the plain push for particles that fail it
 * (to help, it should be at least as accurate as the network's step; for a
 * network with a base push that means more substeps than the base push).
 * ep_step then needs a 5-input network for the Duffing field and a 6-input
 * one for the Poisson field; the base push and the energy projection of the
 * loaded network and context apply (see the learned section below).
 * Errors: EP_EINVAL, EP_ENOTRAINED. */
ep_status ep_set_push_mode(ep_ctx *ctx, int32_t push, double drift_tol,
                           uint32_t fallback_substeps);

/* ---------------------------------------------------------------- fine solvers
 * EP_PUSH_RK4: each macro step dt is K = ceil(dt / h_fine) classic RK4 steps
 * of size dt / K on y' = (1/eps) M y + (0, E(t, R)) (eq. 1.4, FP64 in the lab
 * frame); for the Poisson field all particles advance together and the
 * charge is deposited and the mesh solved again at every stage.
 * EP_PUSH_IMPROVED_ETD: each macro step is Algorithm 3.4 — per-particle
 * periods T_i (time between the first and third sign change of V along a
 * fine RK4 solve from y^n; Remark 3.5), dt = N_i T_i + o_i, a second fine
 * solve from y^n giving y(t_n + o_i) and y(t_n + o_i + T_i) by quadratic
 * interpolation through three fine levels (Remark 3.6), and
 * y^{n+1} = y(t_n + o_i) + N_i (y(t_n + o_i + T_i) - y(t_n + o_i)) (Lemma 3.3).
 * EP_PUSH_CLASSIC_ETD / EP_PUSH_MODIFIED_ETD: Algorithm 2.1 with a common
 * period P (2 pi eps, or the mean of the periods T_i found as above):
 * dt = N P + o, y(t_n + P) by ceil(P / h_fine) equal RK4 steps, y(t_n + N P) =
 * y^n + N (y(t_n + P) - y^n), then ceil(o / h_fine) equal steps over o.
 * h_fine <= 0 selects the paper's fine step 2 pi eps / 100 at each ep_step.
 * max_fine (>= 1) bounds the fine steps of the period search; a particle
 * without three sign changes by then keeps the free period 2 pi eps and is
 * counted as unresolved.  The sorted deposit does not support these modes.
 * periods_once (0 or 1): in the Duffing field each particle's period is
 * constant (section 3), so with periods_once = 1 an improved ETD step reuses
 * the periods found by the preceding improved ETD, modified ETD or
 * ep_compute_periods call on the same particles, with the same eps and fine
 * step, when no other step came in between; it then runs only the capture
 * solve, and ep_get_periods keeps reporting the unresolved count of the
 * search that found them.  The self-consistent field searches at every step.
 * Calling ep_set_fine_solver drops the kept periods.
 * Defaults: h_fine = 0, max_fine = 10000, periods_once = 1.  Errors:
 * EP_EINVAL. */
ep_status ep_set_fine_solver(ep_ctx *ctx, double h_fine, uint64_t max_fine,
                             int32_t periods_once);

/* The periods T_i of the current state, without stepping (the paper's period
 * diagnostics, section 2): the same fine-solve search as Algorithm 3.4 uses,
 * for the Duffing or the Poisson field; ep_get_periods then returns them with
 * N_i = 0.  Errors: EP_EINVAL, EP_ESTATE, EP_ENOMEM, EP_EHIP. */
ep_status ep_compute_periods(ep_ctx *ctx, double eps, int32_t field, uint64_t *n_unresolved);

/* After an EP_PUSH_IMPROVED_ETD or EP_PUSH_MODIFIED_ETD step: the periods
 * T_i (FP64) and whole numbers of periods N_i (the common N for the modified
 * scheme) used by the last macro step, for particles
 * [offset, offset + count) in loaded order, and the number of unresolved
 * particles of that step (any output may be NULL).  Synchronises.
 * Errors: EP_EINVAL, EP_ESTATE (no such step yet), EP_EHIP. */
ep_status ep_get_periods(ep_ctx *ctx, double *T, int64_t *N, uint64_t offset, uint64_t count,
                         uint64_t *n_unresolved);

/* ---------------------------------------------------------------- learned
 * Learned Duhamel corrector: a 5 -> 64 -> 64 -> 2 network (6 inputs for the
 * Poisson field) with the activation z / sqrt(1 + z^2).  Features of a
 * particle y = (R, V) for a step dt at eps:
 *   (R / s_in, V / s_in, cos phi, sin phi, (dt/eps) / s_t [, E^n(R) / s_E]),
 *   phi = (dt/eps) mod 2 pi.
 * Its outputs o give the step's Duhamel term (eq. 3.6) in polar form around
 * the exact rotation: delta = mu_d + sig_d o_0, kappa = mu_k + sig_k o_1 and
 *   y_{n+1} = (1 + kappa) r(dt/eps + delta) y_n.
 * With the amplitude-scaled output map the two outputs are a delta and
 * a kappa (a = |y_n|: the arc length and the radial displacement beyond the
 * free rotation), divided by a before the map is applied; they stay bounded
 * for small orbits in the self-consistent field, whose phase advance grows
 * like 1/a.  Base push (Duffing field, 5-input network): with K_b > 0 the
 * same polar map acts around the plain push of y_n with K_b substeps,
 *   y_{n+1} = (1 + kappa) r(delta) y_b,  y_b = plain K_b-substep step of y_n,
 * so that the network predicts that push's defect against the fine push, a
 * correction that shrinks like K_b^-2; each learned step then runs the base
 * push (every particle, FP64, result stored in FP32) before the network.
 * Training labels follow the map and the base of the loaded normalisation.
 * Parameters: one FP32 vector W1[64][n_in], b1[64], W2[64][64], b2[64],
 * W3[2][64], b3[2] (row-major; 4674 values for n_in = 5, 4738 for 6).
 * Normalisation: 9 doubles {s_in, s_t, s_E, mu_d, sig_d, mu_k, sig_k, map,
 * K_b}, map = 0 (delta, kappa) or 1 (amplitude-scaled), K_b = 0 (around the
 * free rotation) or the base push's substeps (a whole number <= 4096). */
typedef struct {
    double dt, eps;            /* step the corrector is trained for (> 0)            */
    int32_t field;             /* EP_FIELD_DUFFING (given samples) or EP_FIELD_POISSON
                                  (samples collected with ep_mlp_collect)           */
    uint32_t fine_substeps;    /* K of the plain push that makes the labels (>= 1)  */
    uint32_t batch;            /* samples per Adam step, a multiple of 64            */
    uint32_t epochs;           /* passes over the samples (>= 1)                     */
    double lr, lr_final;       /* Adam step size, cosine-decayed from lr to lr_final */
    double s_in;               /* feature scale of R and V (> 0)                     */
} ep_train_cfg;

typedef struct {
    uint64_t steps;            /* Adam steps taken                                   */
    double loss_first;         /* mean loss (normalised labels) of the first epoch   */
    double loss_last;          /* mean loss of the last epoch                        */
    double mu_delta, sig_delta, mu_kappa, sig_kappa;  /* label normalisation         */
    double label_ms, train_ms; /* GPU time of label generation and of training       */
} ep_train_report;

/* MFMA operand type of the learned push (the inference; training always uses
 * BF16 products with FP32 accumulation). */
typedef enum {
    EP_MLP_BF16 = 0, /* default: layer-1 weights and features as split BF16
                        (hi + lo), W2 and W3 as split BF16, activations computed
                        in FP32 and rounded to BF16                             */
    EP_MLP_FP16 = 1  /* layer-1 weights and features as split FP16, W2 and W3 in
                        FP16, activations in packed FP16 arithmetic: faster and
                        closer to the FP64 network; networks whose pre-
                        activations could reach |z| >= 16320 are refused with
                        EP_EINVAL by the step that needs them                   */
} ep_mlp_precision;

/* Select the inference operand type (ep_mlp_precision) for later learned
 * steps.  Errors: EP_EINVAL (unknown value). */
ep_status ep_mlp_set_precision(ep_ctx *ctx, int32_t precision);

/* Energy projection of the learned push (on = 1; default 0).  The exact step
 * conserves the energy H^n = |y|^2/(2 eps) + P(R) of the energy check (the
 * Duffing energy, a first integral of eq. 1.4 with E = -r^3 (appendix A), or
 * the frozen-field energy of the step), which the network's map does only
 * to its fit, with errors that share a sign and add up over long runs.  With
 * the projection every particle of the step (the network's after the check,
 * and the fallback's) is moved radially back onto its energy shell by one
 * Newton step from s = 1 of H^n(s y_{n+1}) = H^n(y_n):
 * s = 1 - (H^n(y_{n+1}) - H^n(y_n)) / S,
 * S = |y_{n+1}|^2 / eps + R_{n+1} P'(R_{n+1}), skipped where S is not above
 * half of |y_{n+1}|^2 / eps; the phase of the result is kept and the check
 * decides on the unprojected prediction.  A setting of the context
 * (kept across networks, saved in checkpoints).  Errors: EP_EINVAL. */
ep_status ep_mlp_set_projection(ep_ctx *ctx, int32_t on);

/* Load network parameters (n_params = 4674 or 4738 FP32 values, layout above)
 * and their normalisation (9 doubles).  Errors: EP_EINVAL (also for K_b > 0
 * with a 6-input network). */
ep_status ep_mlp_set_weights(ep_ctx *ctx, const float *params, uint32_t n_params,
                             const double *norm);

/* Copy the current parameters and normalisation (9 doubles) out.  n_params
 * must match.
 * Errors: EP_EINVAL, EP_ENOTRAINED, EP_EHIP. */
ep_status ep_mlp_get_weights(ep_ctx *ctx, float *params, uint32_t n_params, double *norm);

/* Training labels: for n samples (R, V) (host FP64, rounded to FP32 like the
 * features), one plain step of dt at eps with K fine substeps in the Duffing
 * field, returned in polar form delta[n], kappa[n] (FP32): the phase advance
 * beyond the free rotation and the relative change of |y|, or, if the loaded
 * network has a base push, the same from the base push's result.
 * Errors: EP_EINVAL, EP_EHIP. */
ep_status ep_mlp_labels(ep_ctx *ctx, double dt, double eps, uint32_t fine_substeps,
                        const double *R, const double *V, uint64_t n, float *delta,
                        float *kappa);

/* Gradient of the loss mean((o - (y - mu)/sig)^2) over a batch (X[batch][n_in]
 * features, Y[batch][2] raw labels (delta, kappa); mu, sig from the current
 * normalisation) at the current parameters, as computed by the training
 * kernels (BF16 MFMA products, FP32 accumulation).  grad has n_params entries.
 * Errors: EP_EINVAL, EP_ENOTRAINED, EP_EHIP. */
ep_status ep_mlp_grad(ep_ctx *ctx, const float *X, const float *Y, uint32_t batch, float *grad,
                      double *loss);

/* Self-generated training samples for the Poisson field (6-input network):
 * from the context's particles first, first + stride, ... at the current time
 * level and its field E^n (computed first if stale), the features
 * (R/s_in, V/s_in, cos phi, sin phi, (dt/eps)/s_t, E^n(R)/s_E), with the
 * scales of the loaded normalisation, and the labels (delta, kappa) of one
 * plain step of dt at eps with fine_substeps substeps in the frozen field E^n
 * (the standard PIC field time level).  The samples are appended to the
 * context's training set (cleared first if reset != 0); *n_total receives its
 * size.  Changing the network's input count discards the set.
 * Errors: EP_EINVAL, EP_ENOTRAINED, EP_ESTATE, EP_ENOMEM, EP_EHIP. */
ep_status ep_mlp_collect(ep_ctx *ctx, double dt, double eps, uint32_t fine_substeps,
                         uint64_t first, uint64_t stride, int32_t reset, uint64_t *n_total);

/* Copy rows [first, first + count) of the collected training set out:
 * X[count][6] features, Y[count][2] raw labels (delta, kappa).
 * Errors: EP_EINVAL, EP_EHIP. */
ep_status ep_mlp_get_samples(ep_ctx *ctx, uint64_t first, uint64_t count, float *X, float *Y);

/* Train the network on the GPU, starting from the parameters loaded with
 * ep_mlp_set_weights.  Duffing field: labels of the n samples (R, V) are made
 * with the plain push (cfg->fine_substeps) and batches are taken in sample
 * order; the feature scales become {cfg->s_in, 100, 1}.  Poisson field: R, V
 * and n are ignored, the collected set is used (feature scales unchanged), and
 * batch b of an epoch takes the rows b, b + P, b + 2P, ... (P batches per
 * epoch), so that each batch spans all collected time levels.  The
 * normalisation of the labels is set from the mean and standard deviation of
 * the first 65536 labels; Adam runs cfg->epochs passes with a step size
 * cosine-decayed from lr to lr_final.  Errors: EP_EINVAL, EP_ENOTRAINED,
 * EP_ENOMEM, EP_EHIP. */
ep_status ep_mlp_train(ep_ctx *ctx, const ep_train_cfg *cfg, const double *R, const double *V,
                       uint64_t n, ep_train_report *report);

/* ---------------------------------------------------------------- checkpoint
 * ep_save writes the state of the current time level to `path`: a header
 * (magic "ETDPIC01", format version, loaded particle count, mesh and substep
 * configuration, weight, t, phase, step count, push mode, fallback settings,
 * inference precision, fine-solver settings),
 * the FP32 rotating-frame particle arrays in the order they were loaded, the
 * corrector's parameters and normalisation if one is loaded, and the periods
 * T_i and N_i of the last improved or modified ETD step (or ep_compute_periods
 * call) if they belong to the saved particles, so that a resumed improved ETD
 * run reuses them as the uninterrupted run does.  ep_load
 * restores such a file into a context whose capacity, mesh and substeps
 * accept it; the field is recomputed from the particles, so a resumed run
 * continues bit for bit.  A push mode the context cannot run (the learned
 * push without a network, a fine solver with the sorted deposit) is restored
 * as the plain push.  The fallback counter of ep_moments is a statistic,
 * not state: it is not saved.  Errors: EP_EIO (file cannot be opened, read or
 * written, or is not a checkpoint of this format), EP_EINVAL (it does not fit
 * the context), EP_EHIP.  ep_load stores the restored particle count in
 * *n_particles when that pointer is not null. */
ep_status ep_save(ep_ctx *ctx, const char *path);
ep_status ep_load(ep_ctx *ctx, const char *path, uint64_t *n_particles);

/* Achieved bandwidth of a plain device-to-device copy of `bytes` on `device`
 * (reps timed copies after 3 untimed ones), counting bytes read plus bytes
 * written: a practical ceiling to compare the particle kernels with.  Needs
 * no context; allocates and frees two buffers of `bytes`.
 * Errors: EP_EINVAL, EP_ENOMEM, EP_EHIP. */
ep_status ep_copy_bandwidth(int32_t device, uint64_t bytes, int32_t reps, double *gb_per_s);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the plain
 * step of ep_step without a context.  zR[n], zV[n] are the caller's FP32
 * device arrays (16-byte aligned) holding the rotating-frame state
 * z = r(-phase) y at the host value *phase = t/eps mod 2 pi, with uniform
 * weight w > 0.  n_steps macro steps of dt at eps in the field model `field`
 * are queued on hip_stream (NULL: the null stream), and *phase receives the
 * phase after them.  The Poisson field is first deposited from the current
 * state and solved, as a fresh context does, on a mesh of n_cells cells on
 * [-r_max, r_max].  The kernels, their launch order and their arguments are
 * those of ep_step with the atomic deposit, so results equal a context's
 * (bitwise while n_steps * substeps fits the coefficient table, else within
 * the plain push's per-particle tolerance for the Duffing field, whose
 * register-resident launches then store the FP32 state more often).
 * The call allocates nothing: the mesh and the coefficient tables live in
 * one static device array of about 1.8 MB that each device holds until the
 * process ends.  Limits of that array: n_cells <= 8192, substeps <= 32768.
 * Calls on the same device share it, so calls whose work overlaps on one GPU
 * (other host threads, or other streams) race; calls queued on one stream do
 * not.  Errors: EP_EINVAL (a limit above, n >= 2^31, bad arguments; the
 * message says which; ep_last_error(NULL) returns it), EP_EHIP (a launch
 * failed; asynchronous kernel errors surface at the caller's next
 * synchronisation of hip_stream). */
ep_status ep_step_noalloc(float *zR, float *zV, uint64_t n, double w, uint32_t n_cells,
                          double r_max, uint32_t substeps, double dt, double eps, int32_t field,
                          uint64_t n_steps, double *phase, int32_t device, void *hip_stream);

/* Synchronise the context's stream; reports asynchronous errors. */
ep_status ep_sync(ep_ctx *ctx);

/* Per-kernel timing with HIP events attached to the launches of the particle
 * kernels on the context's stream.  ep_timing_enable(ctx, on) clears the
 * table and sets the collection: on = 0 stops it, on = 1 times every launch,
 * on = n > 1 every n-th launch of each kernel (the first, the (n+1)-th, ...),
 * which keeps the events' own cost (a few microseconds per timed launch)
 * out of most steps.  ep_timing_get synchronises and returns, for the kernel
 * named `kernel` ("push_poisson", "deposit", "mesh_solve", "push_duffing",
 * "base_push", "mlp_push", "fallback_push",
 * "sort_count", "sort_offsets", "sort_scatter", "sort_combine"), the summed
 * duration in milliseconds and the number of timed launches.
 * Errors: EP_EINVAL (also for on < 0). */
ep_status ep_timing_enable(ep_ctx *ctx, int32_t on);
ep_status ep_timing_get(ep_ctx *ctx, const char *kernel, double *total_ms, uint64_t *count);

#ifdef __cplusplus
}
#endif

#endif /* ETDPIC_H */
