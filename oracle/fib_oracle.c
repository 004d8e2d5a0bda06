/*
 * fib_oracle.c -- plain FP64 CPU oracle for the Strang-split monodomain solve
 * on many independent 1D muscle fibers (Maier, "Scalable Biophysical
 * Simulations of the Neuromuscular System", 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may build, load
 * or call it.  It shares no code, header or table with the GPU library.
 *
 * Everything is double precision, scalar loops, no fast-math.  Each function
 * names the passage of the thesis it follows:
 *   - subcellular model: section "Subcellular Model", eqs. subcellular_model_
 *     helper3-5 and subcellular; the Hodgkin-Huxley rate functions in the
 *     -75 mV resting-potential convention fixed by the generated-code excerpt
 *     in section "Computation of CellML Models" (Hodgkin & Huxley 1952); the
 *     same membrane with exp replaced by the exp* of eq. apx-e-function;
 *   - monodomain equation on a fiber: eq. monodomain, no-flux ends
 *     eq. monodomain_bc1;
 *   - operator splitting: eq. monodomain_strang (0D, 1D, 0D order, figure
 *     splitting_schemes), eq. monodomain_godunov;
 *   - time stepping: eq. heun (0D); the theta-scheme of eq. crank_nicolson
 *     (1D), theta = 1/2 Crank-Nicolson, theta = 1 implicit Euler
 *     (eq. implicit_euler, lumped as in eq. lumping_implicit_euler);
 *   - 1D linear finite elements: tables stencils_laplace and
 *     stencils_mass_laplace, mass lumping (section "Using Mass Lumping for
 *     Implicit Timestepping", eq. lumping_crank_nicolson);
 *   - block-diagonal per-fiber system: eq. discretized_fibers_1;
 *   - Thomas algorithm: section "Improved Parallel Solver Scheme using the
 *     Thomas Algorithm";
 *   - stimulation of the nodes around a neuromuscular junction: section
 *     "Specification of Stimulation Times Using Callback Functions", either
 *     as an injected current or as a prescribed membrane voltage.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

/* ------------------------------------------------------------------------ */
/* Parameters                                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t model;   /* 0: Hodgkin-Huxley (4 states), 1: ST57 (57 states),
                      2: Hodgkin-Huxley with exp* (eq. apx-e-function) */
  int32_t scheme;  /* 0: Strang  R(dt/2) D(dt) R(dt/2);  1: Godunov R(dt) D(dt) */
  double Cm;       /* membrane capacitance, uF/cm^2 */
  double Am;       /* surface-to-volume ratio, 1/cm */
  double sigma;    /* effective conductivity along the fiber, mS/cm */
  double h;        /* node spacing, cm */
  double dt_0D;    /* largest reaction substep, ms */
  double dt_1D;    /* largest diffusion substep, ms */
  double dt_split; /* splitting step, ms */
  double v_th;     /* activation threshold for the activation-time observable, mV */
  double theta;    /* 1D time stepping (eq. crank_nicolson): 0.5 Crank-Nicolson,
                      1 implicit Euler (eq. implicit_euler); values in [0.5, 1] */
} or_params;

typedef struct {
  int32_t fiber;      /* fiber index */
  int32_t node;       /* centre node j (0-based, within the fiber) */
  int32_t half_width; /* nodes j-hw .. j+hw are stimulated (clipped to the fiber) */
  int32_t mode;       /* 0: current density `amp`; 1: V_m prescribed to `amp` */
  int64_t step_on;    /* first split step with the stimulus on */
  int64_t n_steps;    /* number of consecutive split steps with the stimulus on */
  int64_t period;     /* 0: one pulse; >0: the pulse repeats every `period` steps */
  double amp;         /* current density in uA/cm^2 (mode 0) or voltage in mV (mode 1) */
} or_stim;

/* ------------------------------------------------------------------------ */
/* Hodgkin-Huxley membrane (section "Subcellular Model")                     */
/* ------------------------------------------------------------------------ */

#define HH_ER (-75.0)
#define HH_GNA 120.0
#define HH_GK 36.0
#define HH_GL 0.3
#define HH_ENA (HH_ER + 115.0)
#define HH_EK (HH_ER - 12.0)
#define HH_EL (HH_ER + 10.613)

/* The approximate exponential of eq. apx-e-function,
 *   exp*(x) = (1 + x/n)^n  with n = 1024 = 2^10,
 * evaluated as the thesis does: one division by n, one addition and ten
 * squarings. */
double or_exp_star(double x) {
  double u = 1.0 + x / 1024.0;
  for (int i = 0; i < 10; ++i) u *= u;
  return u;
}

/* The approximate logarithm of section "Evaluation of Code Generator
 * Optimizations" (figure apxlog): the sixth-order Taylor polynomial of log
 * around a = 1 for x < 2, around a = 3 for 2 <= x < 6 and around a = 9 for
 * x >= 6,
 *   log a + sum_{k=1..6} (-1)^(k+1) u^k / k,   u = (x - a) / a,
 * stated for 0.2 <= x <= 20. */
double or_log_star_taylor(double x) {
  const double a = x < 2.0 ? 1.0 : (x < 6.0 ? 3.0 : 9.0);
  const double u = (x - a) / a;
  double s = 0.0, p = 1.0;
  for (int k = 1; k <= 6; ++k) {
    p *= u;
    s += (k % 2 ? p : -p) / (double)k;
  }
  return log(a) + s;
}

/* log*(x): the Taylor value y followed by one Newton step on exp*(y) = x
 * with the derivative taken as exp*(y), i.e. y - (1 - x / exp*(y)), which
 * makes log* the inverse of exp* (eq. apx-e-function) up to the step's
 * quadratic remainder.  Reading: arguments outside [0.2, 20], where the
 * polynomials are not meant to be used, are first brought into it by an
 * exact power-of-two scaling, log x = log(x 2^-k) + k log 2.  NaN for
 * x <= 0. */
double or_log_star(double x) {
  if (!(x > 0.0) || isinf(x)) return NAN;
  int k = 0;
  double m = x;
  while (m >= 20.0) { m *= 0.5; ++k; }
  while (m < 0.2) { m *= 2.0; --k; }
  double y = or_log_star_taylor(m);
  y -= 1.0 - m / or_exp_star(y);
  return y + (double)k * log(2.0);
}

/* x / (exp(x) - 1), the shape of alpha_m and alpha_n; removable singularity
 * at x = 0 where the value is 1.  Near 0 the Taylor series 1 - x/2 + x^2/12
 * is used (its truncation error x^4/720 is below 1e-18 for |x| < 1e-4).
 * With apx, exp is exp*: (1 + x/n)^n - 1 = x + a' x^2 + b' x^3 + ... with
 * a' = (n-1)/(2n), b' = (n-1)(n-2)/(6 n^2), so the quotient is
 * 1 - a' x + (a'^2 - b') x^2 + O(x^3) near 0. */
double or_x_over_expm1(int apx, double x) {
  if (!apx) {
    if (fabs(x) < 1e-4) return 1.0 - 0.5 * x + x * x / 12.0;
    return x / expm1(x);
  }
  const double n = 1024.0, a = (n - 1.0) / (2.0 * n), b = (n - 1.0) * (n - 2.0) / (6.0 * n * n);
  if (fabs(x) < 1e-4) return 1.0 - a * x + (a * a - b) * x * x;
  return x / (or_exp_star(x) - 1.0);
}

static double hh_exp(int apx, double x) { return apx ? or_exp_star(x) : exp(x); }

/* Rate constants (1/ms) of the three gates at membrane voltage V (mV).
 * With v = V - E_R the classic forms are
 *   alpha_m = 0.1 (25-v)/(exp((25-v)/10)-1),  beta_m = 4 exp(-v/18),
 *   alpha_h = 0.07 exp(-v/20),                beta_h = 1/(exp((30-v)/10)+1),
 *   alpha_n = 0.01 (10-v)/(exp((10-v)/10)-1), beta_n = 0.125 exp(-v/80);
 * with apx every exp is the exp* of eq. apx-e-function. */
static void hh_rates(int apx, double V, double ab[6]) {
  double v = V - HH_ER;
  ab[0] = or_x_over_expm1(apx, (25.0 - v) / 10.0);
  ab[1] = 4.0 * hh_exp(apx, -v / 18.0);
  ab[2] = 0.07 * hh_exp(apx, -v / 20.0);
  ab[3] = 1.0 / (hh_exp(apx, (30.0 - v) / 10.0) + 1.0);
  ab[4] = 0.1 * or_x_over_expm1(apx, (10.0 - v) / 10.0);
  ab[5] = 0.125 * hh_exp(apx, -v / 80.0);
}

void or_hh_gate_rates(double V, double ab[6]) { hh_rates(0, V, ab); }
void or_hh_apx_gate_rates(double V, double ab[6]) { hh_rates(1, V, ab); }

/* Ionic current density I_ion (uA/cm^2), eq. subcellular_model_helper5 with
 * g_Na = gbar_Na m^3 h and g_K = gbar_K n^4. */
double or_hh_iion(const double y[4]) {
  double V = y[0], m = y[1], h = y[2], n = y[3];
  double gna = HH_GNA * m * m * m * h;
  double gk = HH_GK * n * n * n * n;
  return gna * (V - HH_ENA) + gk * (V - HH_EK) + HH_GL * (V - HH_EL);
}

/* Right-hand side G(y) of the subcellular model, eq. subcellular:
 *   Cm dV/dt = -I_ion + I_stim           (eq. subcellular_model_helper3)
 *   dy/dt    = alpha (1 - y) - beta y    for y in {m, h, n}. */
static void hh_rhs(int apx, double Cm, const double y[4], double I_stim, double dydt[4]) {
  double ab[6];
  hh_rates(apx, y[0], ab);
  dydt[0] = (-or_hh_iion(y) + I_stim) / Cm;
  dydt[1] = ab[0] * (1.0 - y[1]) - ab[1] * y[1];
  dydt[2] = ab[2] * (1.0 - y[2]) - ab[3] * y[2];
  dydt[3] = ab[4] * (1.0 - y[3]) - ab[5] * y[3];
}

void or_hh_rhs(double Cm, const double y[4], double I_stim, double dydt[4]) {
  hh_rhs(0, Cm, y, I_stim, dydt);
}

/* The same membrane with exp replaced by exp* (eq. apx-e-function). */
void or_hh_apx_rhs(double Cm, const double y[4], double I_stim, double dydt[4]) {
  hh_rhs(1, Cm, y, I_stim, dydt);
}

/* Steady-state ionic current with every gate at its equilibrium
 * y_inf = alpha / (alpha + beta) (the frozen-voltage limit of the gate ODE). */
static double hh_iss(int apx, double V) {
  double ab[6], y[4];
  hh_rates(apx, V, ab);
  y[0] = V;
  y[1] = ab[0] / (ab[0] + ab[1]);
  y[2] = ab[2] / (ab[2] + ab[3]);
  y[3] = ab[4] / (ab[4] + ab[5]);
  return or_hh_iion(y);
}

/* Resting state of the membrane: the voltage where the steady-state current
 * vanishes, found by bisection on [-80, -70] mV (I_ss changes sign there)
 * followed by secant polishing; gates at their equilibria. */
static int hh_rest(int apx, double y[4]) {
  double lo = -80.0, hi = -70.0, flo = hh_iss(apx, lo), fhi = hh_iss(apx, hi);
  if (!(flo < 0.0 && fhi > 0.0)) return OR_EINVAL;
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi), fm = hh_iss(apx, mid);
    if (fm == 0.0) { lo = hi = mid; break; }
    if (fm < 0.0) lo = mid; else hi = mid;
    if (hi - lo < 1e-15) break;
  }
  double V = 0.5 * (lo + hi);
  double ab[6];
  hh_rates(apx, V, ab);
  y[0] = V;
  y[1] = ab[0] / (ab[0] + ab[1]);
  y[2] = ab[2] / (ab[2] + ab[3]);
  y[3] = ab[4] / (ab[4] + ab[5]);
  return OR_OK;
}

int or_hh_rest(double y[4]) { return hh_rest(0, y); }
int or_hh_apx_rest(double y[4]) { return hh_rest(1, y); }

/* ------------------------------------------------------------------------ */
/* Model dispatch                                                            */
/* ------------------------------------------------------------------------ */

/* ST57, the 57-state Shorten-type stand-in (st57_oracle.c), exact and with
 * exp* / log* */
int or_st57_n_states(void);
void or_st57_rhs(double Cm, const double* y, double I, double* dydt);
void or_st57_apx_rhs(double Cm, const double* y, double I, double* dydt);

/* Models: 0 Hodgkin-Huxley, 1 ST57, 2 Hodgkin-Huxley with exp* in its
 * rates (eq. apx-e-function), 3 ST57 with every exp replaced by exp* and
 * every log by log*. */
int or_n_states(int model) {
  if (model == 0 || model == 2) return 4;
  if (model == 1 || model == 3) return or_st57_n_states();
  return -1;
}

static void model_rhs(int model, double Cm, const double* y, double I, double* dydt) {
  if (model == 1)
    or_st57_rhs(Cm, y, I, dydt);
  else if (model == 3)
    or_st57_apx_rhs(Cm, y, I, dydt);
  else
    hh_rhs(model == 2, Cm, y, I, dydt);
}

/* ------------------------------------------------------------------------ */
/* Heun's method, eq. heun                                                   */
/* ------------------------------------------------------------------------ */

#define OR_MAX_STATES 64

/* One Heun step of width tau on one node:
 *   y+ = y + tau/2 (G(y) + G(y + tau G(y))). */
static void heun_step(int model, int S, double Cm, double* y, double I, double tau) {
  double k1[OR_MAX_STATES], k2[OR_MAX_STATES], yt[OR_MAX_STATES];
  model_rhs(model, Cm, y, I, k1);
  for (int k = 0; k < S; ++k) yt[k] = y[k] + tau * k1[k];
  model_rhs(model, Cm, yt, I, k2);
  for (int k = 0; k < S; ++k) y[k] = y[k] + 0.5 * tau * (k1[k] + k2[k]);
}

/* Number of equal reaction substeps that cover `span` with width <= dt_0D. */
int64_t or_n_substeps(double span, double dt) {
  int64_t n = (int64_t)ceil(span / dt - 1e-9);
  return n < 1 ? 1 : n;
}

/* Reaction part over `span` for nodes [i0, i1) of the SoA state
 * y[k * n_total + i]: n_sub equal Heun substeps per node, stimulus current
 * I[i] held constant over the span. */
static void reaction_range(const or_params* p, int S, double* y, int64_t n_total,
                           int64_t i0, int64_t i1, const double* I, double span) {
  int64_t nsub = or_n_substeps(span, p->dt_0D);
  double tau = span / (double)nsub;
  double yn[OR_MAX_STATES];
  for (int64_t i = i0; i < i1; ++i) {
    for (int k = 0; k < S; ++k) yn[k] = y[(int64_t)k * n_total + i];
    for (int64_t s = 0; s < nsub; ++s) heun_step(p->model, S, p->Cm, yn, I ? I[i] : 0.0, tau);
    for (int k = 0; k < S; ++k) y[(int64_t)k * n_total + i] = yn[k];
  }
}

/* ------------------------------------------------------------------------ */
/* Thomas algorithm                                                          */
/* ------------------------------------------------------------------------ */

/* Solves the tridiagonal system
 *   a[i] x[i-1] + d[i] x[i] + c[i] x[i+1] = b[i],  i = 0..n-1
 * (a[0] and c[n-1] are ignored) by a forward elimination sweep and a back
 * substitution sweep, without pivoting.  `work` holds n doubles. */
void or_thomas(int64_t n, const double* a, const double* d, const double* c,
               const double* b, double* x, double* work) {
  if (n <= 0) return;
  double* cp = work;
  double den = d[0];
  cp[0] = (n > 1 ? c[0] : 0.0) / den;
  x[0] = b[0] / den;
  for (int64_t i = 1; i < n; ++i) {
    den = d[i] - a[i] * cp[i - 1];
    cp[i] = (i < n - 1 ? c[i] : 0.0) / den;
    x[i] = (b[i] - a[i] * x[i - 1]) / den;
  }
  for (int64_t i = n - 2; i >= 0; --i) x[i] -= cp[i] * x[i + 1];
}

/* ------------------------------------------------------------------------ */
/* 1D diffusion along one fiber: lumped linear FE + Crank-Nicolson           */
/* ------------------------------------------------------------------------ */

/* Row i of M_L^{-1} K for a fiber of n nodes with spacing h and no-flux ends.
 * Element stiffness (1/h)[-1 1; 1 -1] and element mass (h/6)[2 1; 1 2]
 * (tables stencils_laplace, stencils_mass_laplace) assemble to
 * K = (1/h) tridiag(1, -2, 1) with corner entries -1, and the lumped mass
 * (row sums) is h * diag(1/2, 1, ..., 1, 1/2).  Hence row i of M_L^{-1} K is
 * (wl, -(wl+wr), wr) / h^2 with wl, wr in {0, 1, 2}. */
static void lumped_row(int64_t i, int64_t n, double* wl, double* wr) {
  if (n == 1) { *wl = 0.0; *wr = 0.0; return; }
  if (i == 0) { *wl = 0.0; *wr = 2.0; return; }
  if (i == n - 1) { *wl = 2.0; *wr = 0.0; return; }
  *wl = 1.0; *wr = 1.0;
}

/* One theta-scheme step of width dt on one fiber (eq. crank_nicolson with
 * the lumped mass of eq. lumping_crank_nicolson; theta = 1/2 is
 * Crank-Nicolson, theta = 1 the implicit Euler of eq.
 * lumping_implicit_euler):
 *   (I - theta dt L) V+ = (I + (1 - theta) dt L) V,  L = c M_L^{-1} K,
 * with c = sigma / (Am Cm) (eq. monodomain).  The left-hand matrix is
 * assembled row by row and solved by Thomas. */
static void cn_step(const or_params* p, int64_t n, double* V, double dt,
                    double* a, double* d, double* c, double* b, double* x, double* work) {
  double coef = p->sigma / (p->Am * p->Cm);
  double lam = dt * coef / (p->h * p->h);
  double impl = p->theta * lam, expl = (1.0 - p->theta) * lam;
  for (int64_t i = 0; i < n; ++i) {
    double wl, wr;
    lumped_row(i, n, &wl, &wr);
    double left = (i > 0) ? V[i - 1] : 0.0;
    double right = (i < n - 1) ? V[i + 1] : 0.0;
    /* right-hand side (I + (1 - theta) dt L) V */
    b[i] = V[i] + expl * (wl * left - (wl + wr) * V[i] + wr * right);
    /* left-hand matrix (I - theta dt L) */
    a[i] = -impl * wl;
    d[i] = 1.0 + impl * (wl + wr);
    c[i] = -impl * wr;
  }
  or_thomas(n, a, d, c, b, x, work);
  for (int64_t i = 0; i < n; ++i) V[i] = x[i];
}

/* Diffusion part over `span` on one fiber: equal CN substeps of width
 * <= dt_1D. */
static void diffusion_fiber(const or_params* p, int64_t n, double* V, double span,
                            double* scratch) {
  int64_t m = or_n_substeps(span, p->dt_1D);
  double dt = span / (double)m;
  double *a = scratch, *d = a + n, *c = d + n, *b = c + n, *x = b + n, *w = x + n;
  for (int64_t s = 0; s < m; ++s) cn_step(p, n, V, dt, a, d, c, b, x, w);
}

/* ------------------------------------------------------------------------ */
/* Stimulus                                                                  */
/* ------------------------------------------------------------------------ */

/* True if stimulus entry `s` is on during split step `step`: a pulse of
 * n_steps split steps starting at step_on, repeated every `period` steps when
 * period > 0.  The current is held for the whole split step (both reaction
 * halves). */
static int stim_on(const or_stim* s, int64_t step) {
  if (step < s->step_on || s->n_steps <= 0) return 0;
  int64_t k = step - s->step_on;
  if (s->period > 0) k = k % s->period;
  return k < s->n_steps;
}

/* Stimulus current of every node of fiber f (local node index) at `step`
 * from the current-density entries (mode 0). */
static void fiber_current(int32_t f, int64_t n, const or_stim* stim, int32_t n_stim,
                          int64_t step, double* I) {
  for (int64_t i = 0; i < n; ++i) I[i] = 0.0;
  for (int32_t e = 0; e < n_stim; ++e) {
    const or_stim* s = &stim[e];
    if (s->fiber != f || s->mode != 0 || !stim_on(s, step)) continue;
    for (int64_t j = (int64_t)s->node - s->half_width; j <= (int64_t)s->node + s->half_width; ++j)
      if (j >= 0 && j < n) I[j] += s->amp;
  }
}

/* Prescribed-voltage entries (mode 1) on during `step`: the membrane
 * voltage of their nodes is set to `amp` at the start of the split step
 * (section "Specification of Stimulation Times Using Callback Functions":
 * the callback alters the state vector between steps).  V is the fiber's
 * voltage row. */
static void fiber_prescribe(int32_t f, int64_t n, const or_stim* stim, int32_t n_stim,
                            int64_t step, double* V) {
  for (int32_t e = 0; e < n_stim; ++e) {
    const or_stim* s = &stim[e];
    if (s->fiber != f || s->mode != 1 || !stim_on(s, step)) continue;
    for (int64_t j = (int64_t)s->node - s->half_width; j <= (int64_t)s->node + s->half_width; ++j)
      if (j >= 0 && j < n) V[j] = s->amp;
  }
}

/* ------------------------------------------------------------------------ */
/* Single-phase entry points (for phase-by-phase comparisons)                */
/* ------------------------------------------------------------------------ */

/* Reaction over `span` on every node of the SoA state y[S][n_total] with the
 * per-node current I (nullable: no current). */
int or_reaction(const or_params* p, int64_t n_total, double* y, const double* I, double span) {
  int S = or_n_states(p->model);
  if (S <= 0 || n_total < 0 || !(span > 0.0)) return OR_EINVAL;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_total; ++i) reaction_range(p, S, y, n_total, i, i + 1, I, span);
  return OR_OK;
}

/* Diffusion over `span` on the concatenated membrane voltages of n_fibers
 * fibers (fiber f occupies n_nodes[f] consecutive entries of V). */
int or_diffusion(const or_params* p, int32_t n_fibers, const int32_t* n_nodes, double* V,
                 double span) {
  if (n_fibers < 0 || !(span > 0.0) || !(p->theta >= 0.5 && p->theta <= 1.0)) return OR_EINVAL;
  int64_t* off = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n_fibers + 1));
  if (!off) return OR_ENOMEM;
  off[0] = 0;
  for (int32_t f = 0; f < n_fibers; ++f) {
    if (n_nodes[f] < 1) { free(off); return OR_EINVAL; }
    off[f + 1] = off[f] + n_nodes[f];
  }
  int err = OR_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t f = 0; f < n_fibers; ++f) {
    int64_t n = n_nodes[f];
    double* scratch = (double*)malloc(sizeof(double) * 6 * (size_t)n);
    if (!scratch) { err = OR_ENOMEM; continue; }
    diffusion_fiber(p, n, V + off[f], span, scratch);
    free(scratch);
  }
  free(off);
  return err;
}

/* Per-node stimulus current at split step `step` for the concatenated
 * fibers (I has sum(n_nodes) entries). */
int or_stimulus_current(int32_t n_fibers, const int32_t* n_nodes, const or_stim* stim,
                        int32_t n_stim, int64_t step, double* I) {
  int64_t off = 0;
  for (int32_t f = 0; f < n_fibers; ++f) {
    fiber_current(f, n_nodes[f], stim, n_stim, step, I + off);
    off += n_nodes[f];
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* The splitting loop                                                        */
/* ------------------------------------------------------------------------ */

/* Runs split steps step0 .. step0+n_steps-1 on all fibers.
 *
 * y       SoA state y[k * n_total + i], in/out (k = 0 is V_m in mV).
 * stim    stimulus table (n_stim entries).
 * samples nullable; if sample_every > 0, after every split step n with
 *         (n + 1) % sample_every == 0 the membrane voltage is written to
 *         samples[s * n_total + i], s = (n + 1) / sample_every - 1 - first,
 *         where first = step0 / sample_every counts samples of earlier calls.
 * t_act   nullable, in/out: per node the time (ms) of the first upward
 *         crossing of v_th, linearly interpolated between the ends of the
 *         split step; +inf until it happens.
 *
 * Fibers are independent (eq. discretized_fibers_1 is block diagonal), so
 * each fiber is advanced through all steps on its own. */
int or_run(const or_params* p, int32_t n_fibers, const int32_t* n_nodes, double* y,
           const or_stim* stim, int32_t n_stim, int64_t step0, int64_t n_steps,
           int64_t sample_every, double* samples, double* t_act) {
  int S = or_n_states(p->model);
  if (S <= 0 || n_fibers < 0 || n_steps < 0 || step0 < 0 || !(p->dt_split > 0.0) ||
      !(p->theta >= 0.5 && p->theta <= 1.0))
    return OR_EINVAL;
  int64_t* off = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n_fibers + 1));
  if (!off) return OR_ENOMEM;
  off[0] = 0;
  for (int32_t f = 0; f < n_fibers; ++f) {
    if (n_nodes[f] < 1) { free(off); return OR_EINVAL; }
    off[f + 1] = off[f] + n_nodes[f];
  }
  const int64_t n_total = off[n_fibers];
  const double dt = p->dt_split;
  int err = OR_OK;

#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t f = 0; f < n_fibers; ++f) {
    const int64_t n = n_nodes[f], o = off[f];
    double* buf = (double*)malloc(sizeof(double) * ((size_t)S * n + 9 * (size_t)n));
    if (!buf) { err = OR_ENOMEM; continue; }
    double* yf = buf;               /* SoA state of this fiber, S x n */
    double* I = yf + (size_t)S * n; /* stimulus current */
    double* vprev = I + n;          /* V at the start of the split step */
    double* scratch = vprev + n;    /* 6 n for the CN solve */
    for (int k = 0; k < S; ++k)
      memcpy(yf + (size_t)k * n, y + (int64_t)k * n_total + o, sizeof(double) * n);

    for (int64_t step = step0; step < step0 + n_steps; ++step) {
      /* V at the end of the previous step: the activation test spans the
       * whole step, including a prescription at its start */
      memcpy(vprev, yf, sizeof(double) * n);
      fiber_prescribe(f, n, stim, n_stim, step, yf);
      fiber_current(f, n, stim, n_stim, step, I);
      if (p->scheme == 0) {
        reaction_range(p, S, yf, n, 0, n, I, 0.5 * dt);
        diffusion_fiber(p, n, yf, dt, scratch);
        reaction_range(p, S, yf, n, 0, n, I, 0.5 * dt);
      } else {
        reaction_range(p, S, yf, n, 0, n, I, dt);
        diffusion_fiber(p, n, yf, dt, scratch);
      }
      if (t_act) {
        double t0 = (double)step * dt;
        for (int64_t i = 0; i < n; ++i) {
          double v0 = vprev[i], v1 = yf[i];
          if (isinf(t_act[o + i]) && v0 < p->v_th && v1 >= p->v_th)
            t_act[o + i] = t0 + dt * (p->v_th - v0) / (v1 - v0);
        }
      }
      if (samples && sample_every > 0 && (step + 1) % sample_every == 0) {
        int64_t s = (step + 1) / sample_every - 1 - step0 / sample_every;
        memcpy(samples + s * n_total + o, yf, sizeof(double) * n);
      }
    }
    for (int k = 0; k < S; ++k)
      memcpy(y + (int64_t)k * n_total + o, yf + (size_t)k * n, sizeof(double) * n);
    free(buf);
  }
  free(off);
  return err;
}

/* ------------------------------------------------------------------------ */
/* Adaptive computation (section sec:adaptive_computation_for_fiber_based)   */
/* ------------------------------------------------------------------------ */

/* Point states of the adaptive scheme (figure state_chart). */
#define OR_PT_ACTIVE 0   /* not in equilibrium: solved in the next step */
#define OR_PT_INACTIVE 1 /* in equilibrium: not solved */
#define OR_PT_NEIGHBOR 2 /* a neighbour is active: solved and checked in the next step */

/* Marks every inactive point of a fiber with an active neighbour as
 * "neighbor is active": in one step a point can influence only its two
 * neighbours through the linear-element stencil. */
static void mark_neighbors(int64_t n, uint8_t* pt) {
  for (int64_t i = 0; i < n; ++i) {
    if (pt[i] != OR_PT_INACTIVE) continue;
    if ((i > 0 && pt[i - 1] == OR_PT_ACTIVE) || (i + 1 < n && pt[i + 1] == OR_PT_ACTIVE))
      pt[i] = OR_PT_NEIGHBOR;
  }
}

/* Reaction part over `span` for the points of one fiber that are not
 * inactive (SoA state yf[k * n + i] of the fiber). */
static void reaction_points(const or_params* p, int S, double* yf, int64_t n, const uint8_t* pt,
                            const double* I, double span) {
  int64_t nsub = or_n_substeps(span, p->dt_0D);
  double tau = span / (double)nsub;
  double yn[OR_MAX_STATES];
  for (int64_t i = 0; i < n; ++i) {
    if (pt[i] == OR_PT_INACTIVE) continue;
    for (int k = 0; k < S; ++k) yn[k] = yf[(int64_t)k * n + i];
    for (int64_t s = 0; s < nsub; ++s) heun_step(p->model, S, p->Cm, yn, I[i], tau);
    for (int k = 0; k < S; ++k) yf[(int64_t)k * n + i] = yn[k];
  }
}

/* Equilibrium check of the solved points: moved[i] = 1 if the relative
 * change |y_k - before_k| > tol |before_k| for any state k. */
static void check_points(int S, const double* yf, const double* before, int64_t n,
                         const uint8_t* pt, double tol, uint8_t* moved) {
  for (int64_t i = 0; i < n; ++i) {
    moved[i] = 0;
    if (pt[i] == OR_PT_INACTIVE) continue;
    for (int k = 0; k < S; ++k) {
      const double a = before[(int64_t)k * n + i], b = yf[(int64_t)k * n + i];
      if (fabs(b - a) > tol * fabs(a)) moved[i] = 1;
    }
  }
}

/* Split steps step0 .. step0+n_steps-1 with adaptive computation.  Same
 * arguments and observables as or_run, plus
 *
 * tol       relative change that separates equilibrium from activity;
 * pt        nullable, in/out: per node OR_PT_*; null starts every node
 *           active (the scheme's initial state);
 * computed  nullable, out: number of node-steps whose reaction was solved.
 *
 * Per fiber and split step, in this order:
 *  1. a fiber is left out of the step (neither reaction nor diffusion)
 *     before the first step in which one of its stimulus entries is on
 *     (from the table, whatever step the run starts at); from that step on
 *     it is always part of the computation;
 *  2. V_m prescriptions and currents of the step as in or_run; every point
 *     covered by an entry that is on becomes active, and inactive points
 *     next to an active point become "neighbor is active";
 *  3. the reaction parts of the splitting run on the points that are not
 *     inactive; the diffusion part runs on the whole fiber if any point is
 *     not inactive, else it is skipped;
 *  4. every point solved in the step compares its state before and after
 *     the step's last reaction part (the Heun solve): if the relative change
 *     |y_k+ - y_k| > tol |y_k| for any state k it is active, else inactive;
 *     then inactive points next to an active point become "neighbor is
 *     active" again;
 *  5. observables as in or_run.
 * Points are single nodes (the thesis groups SIMD-vector-sized runs of
 * nodes into one point; the granularity does not enter the definition). */
int or_run_adaptive(const or_params* p, int32_t n_fibers, const int32_t* n_nodes, double* y,
                    const or_stim* stim, int32_t n_stim, int64_t step0, int64_t n_steps,
                    int64_t sample_every, double* samples, double* t_act, double tol,
                    uint8_t* pt, int64_t* computed) {
  int S = or_n_states(p->model);
  if (S <= 0 || n_fibers < 0 || n_steps < 0 || step0 < 0 || !(p->dt_split > 0.0) ||
      !(p->theta >= 0.5 && p->theta <= 1.0) || !(tol >= 0.0))
    return OR_EINVAL;
  int64_t* off = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n_fibers + 1));
  if (!off) return OR_ENOMEM;
  off[0] = 0;
  for (int32_t f = 0; f < n_fibers; ++f) {
    if (n_nodes[f] < 1) { free(off); return OR_EINVAL; }
    off[f + 1] = off[f] + n_nodes[f];
  }
  const int64_t n_total = off[n_fibers];
  const double dt = p->dt_split;
  int err = OR_OK;
  int64_t total = 0;

#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
  for (int32_t f = 0; f < n_fibers; ++f) {
    const int64_t n = n_nodes[f], o = off[f];
    double* buf = (double*)malloc(sizeof(double) * (2 * (size_t)S * n + 9 * (size_t)n));
    uint8_t* ptf = (uint8_t*)malloc(2 * (size_t)n);
    if (!buf || !ptf) { err = OR_ENOMEM; free(buf); free(ptf); continue; }
    uint8_t* moved = ptf + n;
    double* yf = buf;                   /* SoA state of this fiber */
    double* before = yf + (size_t)S * n; /* state before the last reaction part */
    double* I = before + (size_t)S * n;
    double* vprev = I + n;
    double* scratch = vprev + n;
    for (int k = 0; k < S; ++k)
      memcpy(yf + (size_t)k * n, y + (int64_t)k * n_total + o, sizeof(double) * n);
    for (int64_t i = 0; i < n; ++i) ptf[i] = pt ? pt[o + i] : OR_PT_ACTIVE;
    /* first step with a stimulus entry of this fiber on */
    int64_t first_on = INT64_MAX;
    for (int32_t e = 0; e < n_stim; ++e)
      if (stim[e].fiber == f && stim[e].n_steps > 0 && stim[e].step_on < first_on)
        first_on = stim[e].step_on;
    int64_t cnt = 0;

    for (int64_t step = step0; step < step0 + n_steps; ++step) {
      memcpy(vprev, yf, sizeof(double) * n);
      if (step >= first_on) {
        fiber_prescribe(f, n, stim, n_stim, step, yf);
        fiber_current(f, n, stim, n_stim, step, I);
        for (int32_t e = 0; e < n_stim; ++e) {
          const or_stim* s = &stim[e];
          if (s->fiber != f || !stim_on(s, step)) continue;
          for (int64_t j = (int64_t)s->node - s->half_width; j <= (int64_t)s->node + s->half_width; ++j)
            if (j >= 0 && j < n) ptf[j] = OR_PT_ACTIVE;
        }
        mark_neighbors(n, ptf);
        int any = 0;
        for (int64_t i = 0; i < n; ++i) {
          any |= ptf[i] != OR_PT_INACTIVE;
          cnt += ptf[i] != OR_PT_INACTIVE;
        }
        if (p->scheme == 0) {
          reaction_points(p, S, yf, n, ptf, I, 0.5 * dt);
          if (any) diffusion_fiber(p, n, yf, dt, scratch);
          memcpy(before, yf, sizeof(double) * (size_t)S * n);
          reaction_points(p, S, yf, n, ptf, I, 0.5 * dt);
          check_points(S, yf, before, n, ptf, tol, moved);
        } else {
          /* the check compares the ends of the reaction part, before the
           * diffusion changes V */
          memcpy(before, yf, sizeof(double) * (size_t)S * n);
          reaction_points(p, S, yf, n, ptf, I, dt);
          check_points(S, yf, before, n, ptf, tol, moved);
          if (any) diffusion_fiber(p, n, yf, dt, scratch);
        }
        for (int64_t i = 0; i < n; ++i)
          if (ptf[i] != OR_PT_INACTIVE) ptf[i] = moved[i] ? OR_PT_ACTIVE : OR_PT_INACTIVE;
        mark_neighbors(n, ptf);
      }
      if (t_act) {
        double t0 = (double)step * dt;
        for (int64_t i = 0; i < n; ++i) {
          double v0 = vprev[i], v1 = yf[i];
          if (isinf(t_act[o + i]) && v0 < p->v_th && v1 >= p->v_th)
            t_act[o + i] = t0 + dt * (p->v_th - v0) / (v1 - v0);
        }
      }
      if (samples && sample_every > 0 && (step + 1) % sample_every == 0) {
        int64_t s = (step + 1) / sample_every - 1 - step0 / sample_every;
        memcpy(samples + s * n_total + o, yf, sizeof(double) * n);
      }
    }
    for (int k = 0; k < S; ++k)
      memcpy(y + (int64_t)k * n_total + o, yf + (size_t)k * n, sizeof(double) * n);
    if (pt) memcpy(pt + o, ptf, (size_t)n);
    total += cnt;
    free(buf);
    free(ptf);
  }
  free(off);
  if (computed) *computed = total;
  return err;
}
