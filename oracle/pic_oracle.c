/*
 * Plain FP64 CPU oracle of the exponential-integrator PIC step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code, header or constant with the
 * HIP library: every quantity below is written out from the paper's equations.
 *
 * Model (Frenod, Hirstoaga, Lutz, "Long time simulation of a highly oscillatory
 * Vlasov equation with an exponential integrator"):
 *   characteristics  dR/dt = V/eps,  dV/dt = -R/eps + E(R,t)        (eq. 1.4)
 *   stiff linear form y' = (1/eps) M y + L(t,y), M = [[0,1],[-1,0]],
 *                     L = (0, E)                                    (eqs. 3.1-3.2)
 *   rotation          r(tau) = [[cos tau, sin tau], [-sin tau, cos tau]]
 *                     (eq. 3.3 with T = 2*pi, so beta = L in eq. 3.5)
 *   variation of constants over [s, s+h], theta = h/eps           (eq. 3.6)
 *                     y(s+h) = r(theta) y(s)
 *                              + r(theta) Int_s^{s+h} r((s-tau)/eps) L(tau) dtau
 *
 * Push schemes (each is a quadrature of the Duhamel integral of eq. 3.6 with
 * the field frozen over the substep, evaluated along the free rotation):
 *   SCHEME_STRANG : midpoint rule,  y <- r(theta) y + h r(theta/2) (0, E(R_mid)),
 *                   R_mid = [r(theta/2) y]_R          (the hot-path scheme)
 *   SCHEME_ETD1   : exponential Euler, E held at its value at the substep start:
 *                   y <- r(theta) y + eps (1 - cos theta, sin theta) E(R)
 *   SCHEME_ETD2RK : Cox-Matthews second-order exponential Runge-Kutta:
 *                   a = ETD1 step;  y <- a + (eps (1 - sin theta / theta),
 *                   eps (1 - cos theta) / theta) (E(a_R) - E(R))
 *
 * Fields:
 *   FIELD_ZERO    : E = 0 (free rotation with period 2*pi*eps, section 1)
 *   FIELD_DUFFING : E = -R^3 (eq. 1.3)
 *   FIELD_POISSON : d/dr (r E) = rho, rho = Int f dv (eq. 1.2), solved on a
 *                   radial mesh by the trapezoidal rule (section 2.3), with
 *                   cloud-in-cell (CIC) deposit and gather.  Reading of the
 *                   paper for r < 0: E(r) = (1/r) * (1/2) * charge within |r|,
 *                   i.e. the symmetrised enclosed charge, extended oddly.
 *   FIELD_CONST   : E = E0 (test-only field with a closed-form solution)
 *
 * Mesh: nodes x_k = rmin + k*hr, k = 0..nr, hr = (rmax - rmin)/nr, rmin = -rmax,
 * nr even, centre node c = nr/2 at x_c = 0.  A particle is on the mesh iff
 * rmin <= R < rmax; off-mesh particles are not deposited and feel E = Qb / R,
 * where Qb is the half enclosed charge at the mesh edge (Gauss's law).
 *
 * Built with -ffp-contract=off so that every operation rounds as written.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { FIELD_ZERO = 0, FIELD_DUFFING = 1, FIELD_POISSON = 2, FIELD_CONST = 3 };
enum { SCHEME_STRANG = 0, SCHEME_ETD1 = 1, SCHEME_ETD2RK = 2 };

/* ------------------------------------------------------------------ mesh */

typedef struct {
    int nr;         /* number of cells (even)          */
    double rmin;    /* left edge  (= -rmax)            */
    double rmax;    /* right edge                      */
    const double *E;   /* nr+1 node values of E (Poisson) */
    double Qb;         /* half enclosed charge at the edge */
    double E0;         /* constant field (FIELD_CONST)     */
} field_t;

static double mesh_h(int nr, double rmin, double rmax) { return (rmax - rmin) / (double)nr; }

/* CIC charge deposit onto the nr+1 nodes: a particle at R in cell m with
 * fractional offset th gives w(1-th)/hr to node m and w*th/hr to node m+1.
 * rho must hold nr+1 doubles; it is overwritten.  Returns the off-mesh count
 * (NaN positions are counted as off-mesh). */
int64_t orc_deposit(const double *R, int64_t n, double w, int nr, double rmin,
                    double rmax, double *rho)
{
    double hr = mesh_h(nr, rmin, rmax);
    int64_t off = 0;
    for (int k = 0; k <= nr; ++k) rho[k] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double R_i = R[i];
        if (!(R_i >= rmin && R_i < rmax)) { ++off; continue; }
        double s = (R_i - rmin) / hr;
        double m_f = floor(s);
        int m = (int)m_f;
        double th = s - m_f;
        if (m >= nr) { m = nr - 1; th = 1.0; }   /* rounding at the right edge */
        rho[m] += w * (1.0 - th) / hr;
        rho[m + 1] += w * th / hr;
    }
    return off;
}

/* Poisson solve by the trapezoidal rule (section 2.3 of the paper).
 * P_k = Int_{x_0}^{x_k} rho (trapezoid on the node values, exact for the
 * piecewise-linear CIC density), Q_j = (P_{c+j} - P_{c-j}) / 2 (half the charge
 * within |x| <= x_{c+j}), E_{c+-j} = Q_j / x_{c+-j}, E_c = 0.
 * Psi is the potential of E:  Psi_c = 0, Psi' = -E, integrated by the
 * trapezoidal rule on the nodes (exact for the piecewise-linear gathered E).
 * Outputs E[nr+1], Psi[nr+1] (Psi may be NULL), *Qb = Q at the mesh edge. */
void orc_poisson(const double *rho, int nr, double rmin, double rmax,
                 double *E, double *Psi, double *Qb)
{
    double hr = mesh_h(nr, rmin, rmax);
    int c = nr / 2;
    double *P = (double *)malloc(sizeof(double) * (size_t)(nr + 1));
    P[0] = 0.0;
    for (int k = 1; k <= nr; ++k) P[k] = P[k - 1] + hr * (rho[k - 1] + rho[k]) / 2.0;
    E[c] = 0.0;
    for (int j = 1; j <= c; ++j) {
        double Q = (P[c + j] - P[c - j]) / 2.0;
        double x = rmin + (double)(c + j) * hr;
        E[c + j] = Q / x;
        E[c - j] = -Q / x;
    }
    *Qb = (P[nr] - P[0]) / 2.0;
    if (Psi) {
        Psi[c] = 0.0;
        for (int k = c + 1; k <= nr; ++k) Psi[k] = Psi[k - 1] - hr * (E[k - 1] + E[k]) / 2.0;
        for (int k = c - 1; k >= 0; --k) Psi[k] = Psi[k + 1] + hr * (E[k] + E[k + 1]) / 2.0;
    }
    free(P);
}

/* CIC gather of the node field at R; off the mesh, E = Qb / R. */
double orc_gather(double R, const double *E, double Qb, int nr, double rmin, double rmax)
{
    if (!(R >= rmin && R < rmax)) return Qb / R;
    double hr = mesh_h(nr, rmin, rmax);
    double s = (R - rmin) / hr;
    double m_f = floor(s);
    int m = (int)m_f;
    double th = s - m_f;
    if (m >= nr) { m = nr - 1; th = 1.0; }
    return (1.0 - th) * E[m] + th * E[m + 1];
}

/* Potential Psi(R) of the gathered field: -dPsi/dR = E_CIC(R).  Inside cell m
 * E is linear, so Psi is the exact quadratic; off the mesh E = Qb/R gives a
 * logarithm matched to the edge node. */
double orc_potential(double R, const double *E, const double *Psi, double Qb,
                     int nr, double rmin, double rmax)
{
    double hr = mesh_h(nr, rmin, rmax);
    if (R >= rmax) return Psi[nr] - Qb * log(R / rmax);
    if (R < rmin) return Psi[0] - Qb * log(R / rmin);
    if (!(R == R)) return R;
    double s = (R - rmin) / hr;
    double m_f = floor(s);
    int m = (int)m_f;
    if (m >= nr) m = nr - 1;
    double d = R - (rmin + (double)m * hr);
    return Psi[m] - (E[m] * d + (E[m + 1] - E[m]) * d * d / (2.0 * hr));
}

static double field_at(const field_t *f, int kind, double R)
{
    switch (kind) {
    case FIELD_DUFFING: return -R * R * R;
    case FIELD_POISSON: return orc_gather(R, f->E, f->Qb, f->nr, f->rmin, f->rmax);
    case FIELD_CONST: return f->E0;
    default: return 0.0;
    }
}

/* ------------------------------------------------------------------ push */

/* y <- r(phi) y */
static void rotate(double phi, double *R, double *V)
{
    double c = cos(phi), s = sin(phi);
    double r = c * (*R) + s * (*V);
    double v = -s * (*R) + c * (*V);
    *R = r;
    *V = v;
}

/* One macro step dt = K*h of one particle, field frozen (the caller supplies
 * E^n for the Poisson field). */
static void push_one(double *Rp, double *Vp, double dt, double eps, int K, int scheme,
                     int kind, const field_t *f)
{
    double h = dt / (double)K;
    double th = h / eps;
    double R = *Rp, V = *Vp;
    for (int k = 0; k < K; ++k) {
        if (scheme == SCHEME_STRANG) {
            /* midpoint of the Duhamel integral: y_mid = r(theta/2) y */
            double Rm = R, Vm = V;
            rotate(th / 2.0, &Rm, &Vm);
            double E = field_at(f, kind, Rm);
            /* y <- r(theta) y + h r(theta/2) (0, E) */
            double kR = 0.0, kV = h * E;
            rotate(th / 2.0, &kR, &kV);
            rotate(th, &R, &V);
            R = R + kR;
            V = V + kV;
        } else {
            double E = field_at(f, kind, R);
            double aR = R, aV = V;
            rotate(th, &aR, &aV);
            aR = aR + eps * (1.0 - cos(th)) * E;
            aV = aV + eps * sin(th) * E;
            if (scheme == SCHEME_ETD2RK) {
                double dE = field_at(f, kind, aR) - E;
                aR = aR + eps * (1.0 - sin(th) / th) * dE;
                aV = aV + eps * (1.0 - cos(th)) / th * dE;
            }
            R = aR;
            V = aV;
        }
    }
    *Rp = R;
    *Vp = V;
}

/* Push n particles one macro step in a given field (no deposit).  For
 * FIELD_POISSON the node field E[nr+1] and Qb are inputs. */
void orc_push(double *R, double *V, int64_t n, double dt, double eps, int K, int scheme,
              int kind, const double *E, double Qb, int nr, double rmin, double rmax,
              double E0)
{
    field_t f = { nr, rmin, rmax, E, Qb, E0 };
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) push_one(&R[i], &V[i], dt, eps, K, scheme, kind, &f);
}

/* ------------------------------------------------------------------ moments */

/* Diagnostics of the lab-frame state at one time level.
 *  out[0] charge = w * (number of particles)
 *  out[1] rms radius = sqrt(sum w R^2 / sum w)
 *  out[2] energy  = kinetic + potential
 *  out[3] kinetic = sum w (R^2 + V^2) / (2 eps)
 *  out[4] potential: Duffing sum w R^4/4; Poisson Int_0^{rmax} x E^2 dx
 *         (trapezoid on the nodes); zero otherwise
 *  out[5] off-mesh count (Poisson only), out[6] NaN count
 * For the Poisson field E[nr+1] must be the field of these positions. */
void orc_moments(const double *R, const double *V, int64_t n, double w, double eps,
                 int kind, const double *E, int nr, double rmin, double rmax,
                 double *out)
{
    double sR2 = 0.0, sK = 0.0, sP = 0.0;
    int64_t n_off = 0, n_nan = 0;
    for (int64_t i = 0; i < n; ++i) {
        double r = R[i], v = V[i];
        if (!(r == r) || !(v == v) || isinf(r) || isinf(v)) { ++n_nan; continue; }
        sR2 += w * r * r;
        sK += w * (r * r + v * v) / (2.0 * eps);
        if (kind == FIELD_DUFFING) sP += w * r * r * r * r / 4.0;
        if (kind == FIELD_POISSON && !(r >= rmin && r < rmax)) ++n_off;
    }
    if (kind == FIELD_POISSON) {
        double hr = mesh_h(nr, rmin, rmax);
        int c = nr / 2;
        for (int k = c; k < nr; ++k) {
            double x0 = rmin + (double)k * hr, x1 = rmin + (double)(k + 1) * hr;
            sP += hr * (x0 * E[k] * E[k] + x1 * E[k + 1] * E[k + 1]) / 2.0;
        }
    }
    double charge = w * (double)n;
    out[0] = charge;
    out[1] = sqrt(sR2 / charge);
    out[2] = sK + sP;
    out[3] = sK;
    out[4] = sP;
    out[5] = (double)n_off;
    out[6] = (double)n_nan;
}

/* ------------------------------------------------------------------ run */

/* n_steps macro steps of the PIC method.  For FIELD_POISSON each step
 * deposits R^n, solves for E^n, then pushes with E^n frozen over the step.
 * If mom is non-NULL it receives 7 moments per time level, for levels
 * 0..n_steps (so 7*(n_steps+1) doubles). */
void orc_run(double *R, double *V, int64_t n, double w, double dt, double eps, int K,
             int scheme, int kind, int64_t n_steps, int nr, double rmin, double rmax,
             double E0, double *mom)
{
    double *rho = NULL, *E = NULL;
    double Qb = 0.0;
    if (kind == FIELD_POISSON) {
        rho = (double *)malloc(sizeof(double) * (size_t)(nr + 1));
        E = (double *)malloc(sizeof(double) * (size_t)(nr + 1));
    }
    for (int64_t s = 0; s <= n_steps; ++s) {
        if (kind == FIELD_POISSON) {
            orc_deposit(R, n, w, nr, rmin, rmax, rho);
            orc_poisson(rho, nr, rmin, rmax, E, NULL, &Qb);
        }
        if (mom) orc_moments(R, V, n, w, eps, kind, E, nr, rmin, rmax, mom + 7 * s);
        if (s == n_steps) break;
        orc_push(R, V, n, dt, eps, K, scheme, kind, E, Qb, nr, rmin, rmax, E0);
    }
    free(rho);
    free(E);
}

/* Number of OpenMP threads the push would use (1 without OpenMP). */
int orc_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of OpenMP threads of later pushes (n >= 1). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
