/*
 * st57_oracle.c -- FP64 oracle of ST57, the 57-state Shorten-type stand-in
 * subcellular model (the repository's written spec; the thesis's Shorten
 * model itself is not available, so parity against it is unpinned).
 *
 * TEST INFRASTRUCTURE ONLY (see fib_oracle.c).  Plain scalar FP64, written
 * from the specification table, sharing nothing with the GPU library.
 *
 * The model keeps the thesis's Hodgkin-Huxley membrane as states 0-3
 * (section "Subcellular Model") and adds a tubular compartment, a
 * voltage-sensor chain, calcium/magnesium buffering, ion concentrations with
 * Nernst potentials, a Na/K pump cycle, a thin-filament chain, a
 * cross-bridge cycle and two mechanical states, giving the size (57 states)
 * and the mix of exp / log / integer powers / branches the thesis reports
 * for its Shorten model.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define ST_N 57
#define KT 26.71

/* exp*, log* and x / (exp(x) - 1) of fib_oracle.c (the approximations of
 * section "Evaluation of Code Generator Optimizations") */
double or_exp_star(double x);
double or_log_star(double x);
double or_x_over_expm1(int apx, double x);

/* The model's exponential and logarithm: exact, or exp* and log* (apx). */
static double EXP(int apx, double x) { return apx ? or_exp_star(x) : exp(x); }
static double LOG(int apx, double x) { return apx ? or_log_star(x) : log(x); }

/* HH rate constants at voltage V (same forms as the membrane model) */
static void hh_rates(int apx, double V, double* am, double* bm, double* ah, double* bh,
                     double* an, double* bn) {
  double v = V + 75.0;
  *am = or_x_over_expm1(apx, (25.0 - v) / 10.0);
  *bm = 4.0 * EXP(apx, -v / 18.0);
  *ah = 0.07 * EXP(apx, -v / 20.0);
  *bh = 1.0 / (EXP(apx, (30.0 - v) / 10.0) + 1.0);
  *an = 0.1 * or_x_over_expm1(apx, (10.0 - v) / 10.0);
  *bn = 0.125 * EXP(apx, -v / 80.0);
}

int or_st57_n_states(void) { return ST_N; }

/* Conserved sums: sum P, sum Q, sum R, sum X, total Ca (uM), total Mg (uM). */
void or_st57_invariants(const double* y, double out[6]) {
  double s = 0.0;
  for (int i = 8; i <= 17; ++i) s += y[i];
  out[0] = s;
  s = 0.0;
  for (int i = 35; i <= 38; ++i) s += y[i];
  out[1] = s;
  s = 0.0;
  for (int i = 39; i <= 46; ++i) s += y[i];
  out[2] = s;
  s = 0.0;
  for (int i = 47; i <= 54; ++i) s += y[i];
  out[3] = s;
  out[4] = y[18] + y[21] + y[22] + y[24] + 0.1 * (y[19] + y[27]) + 0.01 * (y[20] + y[28]);
  out[5] = y[26] + y[23] + y[25];
}

/* Right-hand side of ST57 with stimulus current I (uA/cm^2); with apx every
 * exp is exp* and every log is log*. */
static void st57_rhs(int apx, double Cm, const double* y, double I, double* d) {
  /* states */
  const double V = y[0], m = y[1], h = y[2], n = y[3];
  const double Vt = y[4], mt = y[5], ht = y[6], nt = y[7];
  const double* P = y + 8;
  const double cm = y[18], cs = y[19], cj = y[20], bT = y[21], bP = y[22], gP = y[23],
               bA = y[24], gA = y[25], gm = y[26], bC = y[27], bCj = y[28];
  const double Nai = y[29], Ki = y[30], Cli = y[31], Nat = y[32], Kt = y[33], Clt = y[34];
  const double* Q = y + 35;
  const double* R = y + 39;
  const double* X = y + 47;
  const double Ls = y[55], gam = y[56];

  /* F: Na/K pump cycle */
  const double k1 = Nai * Nai * Nai / (1000.0 + Nai * Nai * Nai), b1 = 0.05;
  const double k2 = 0.8 * EXP(apx, 0.3 * V / KT), b2 = 0.05;
  const double k3 = 1.2 * Kt * Kt / (2.25 + Kt * Kt), b3 = 0.02;
  const double k4 = 0.6, b4 = 0.01;
  const double J01 = k1 * Q[0] - b1 * Q[1];
  const double J12 = k2 * Q[1] - b2 * Q[2];
  const double J23 = k3 * Q[2] - b3 * Q[3];
  const double J30 = k4 * Q[3] - b4 * Q[0];
  const double Jp = J12;
  d[35] = J30 - J01;
  d[36] = J01 - J12;
  d[37] = J12 - J23;
  d[38] = J23 - J30;

  /* A: surface membrane */
  double am, bm, ah, bh, an, bn;
  hh_rates(apx, V, &am, &bm, &ah, &bh, &an, &bn);
  const double INas = 120.0 * m * m * m * h * (V - 40.0);
  const double IKs = 36.0 * n * n * n * n * (V + 87.0);
  const double ILs = 0.3 * (V + 64.387);
  const double ECl = -KT * LOG(apx, 128.0 / Cli);
  const double IClS = 0.05 * (V - ECl);
  const double Ic = 0.2 * (V - Vt);
  const double Ips = 0.2 * Jp;
  d[0] = (I - (INas + IKs + ILs) - IClS - Ic - Ips) / Cm;
  d[1] = am * (1.0 - m) - bm * m;
  d[2] = ah * (1.0 - h) - bh * h;
  d[3] = an * (1.0 - n) - bn * n;

  /* B: tubular membrane */
  double amt, bmt, aht, bht, ant, bnt;
  hh_rates(apx, Vt, &amt, &bmt, &aht, &bht, &ant, &bnt);
  const double ENa = KT * LOG(apx, Nat / Nai);
  const double EK = KT * LOG(apx, Kt / Ki);
  const double EClt = -KT * LOG(apx, Clt / Cli);
  const double INat = 12.0 * mt * mt * mt * ht * (Vt - ENa);
  const double IKt = 3.6 * nt * nt * nt * nt * (Vt - EK);
  const double IClt = 0.05 * (Vt - EClt);
  const double Ipt = 0.1 * Jp;
  d[4] = (4.0 * 0.2 * (V - Vt) - (INat + IKt + IClt + Ipt)) / Cm;
  d[5] = amt * (1.0 - mt) - bmt * mt;
  d[6] = aht * (1.0 - ht) - bht * ht;
  d[7] = ant * (1.0 - nt) - bnt * nt;

  /* C: voltage-sensor chain driven by Vt */
  double kf[9], kb[9];
  for (int i = 0; i < 9; ++i) {
    const double Vi = -70.0 + 7.5 * i;
    kf[i] = EXP(apx, (Vt - Vi) / 25.0);
    kb[i] = EXP(apx, -(Vt - Vi) / 25.0);
  }
  for (int i = 0; i < 10; ++i) {
    double r = 0.0;
    if (i > 0) r += kf[i - 1] * P[i - 1] - kb[i - 1] * P[i];
    if (i < 9) r += kb[i] * P[i + 1] - kf[i] * P[i];
    d[8 + i] = r;
  }

  /* D: calcium and magnesium */
  const double fload = cj > 500.0 ? 1.0 : cj / 500.0;
  const double Jrel = 1.0 * P[9] * fload * (cj - cm);
  const double Jleak = 2e-5 * (cj - cm);
  const double cplus = cm > 0.0 ? cm : 0.0;
  const double Jup = 4.0 * cplus * cplus / (1.0 + cplus * cplus);
  const double Jtr = 0.02 * (cs - cj);
  const double RT = 0.0885 * cm * (140.0 - bT) - 0.115 * bT;
  const double RP = 0.0417 * cm * (1500.0 - bP - gP) - 5e-4 * bP;
  const double RPM = 3.3e-5 * gm * (1500.0 - bP - gP) - 3e-3 * gP;
  const double RA = 0.15 * cm * (8000.0 - bA - gA) - 30.0 * bA;
  const double RAM = 1.5e-3 * gm * (8000.0 - bA - gA) - 0.15 * gA;
  const double RC = 4e-4 * cs * (31000.0 - bC) - 0.5 * bC;
  const double RCj = 4e-4 * cj * (31000.0 - bCj) - 0.5 * bCj;
  d[18] = Jrel + Jleak - Jup - RT - RP - RA;
  d[19] = (Jup - Jtr) / 0.1 - RC;
  d[20] = (Jtr - Jrel - Jleak) / 0.01 - RCj;
  d[21] = RT;
  d[22] = RP;
  d[23] = RPM;
  d[24] = RA;
  d[25] = RAM;
  d[26] = -RPM - RAM;
  d[27] = RC;
  d[28] = RCj;

  /* E: ion concentrations */
  const double Ip = 0.2 * Jp + 4.0 * 0.1 * Jp;
  d[29] = -2e-5 * (INas + 4.0 * INat + 3.0 * Ip) - (Nai - 10.0) / 1000.0;
  d[30] = -2e-5 * (IKs + 4.0 * IKt - 2.0 * Ip) - (Ki - 140.0) / 1000.0;
  d[31] = 2e-5 * (IClS + 4.0 * IClt) - (Cli - 5.0) / 1000.0;
  d[32] = 2e-3 * (INat + 0.3 * Jp) - (Nat - 140.0) / 50.0;
  d[33] = 2e-3 * (IKt - 0.2 * Jp) - (Kt - 5.0) / 50.0;
  d[34] = -2e-3 * IClt - (Clt - 128.0) / 50.0;

  /* G: thin-filament chain */
  const double th = bT / 140.0;
  const double rf = 2.0 * th * th + 1e-3;
  const double rb = 0.3 / (1.0 + 5.0 * th);
  for (int i = 0; i < 8; ++i) {
    double r = 0.0;
    if (i > 0) r += rf * R[i - 1] - rb * R[i];
    if (i < 7) r += rb * R[i + 1] - rf * R[i];
    d[39 + i] = r;
  }

  /* H: cross-bridge cycle */
  const double a = gA / 8000.0;
  const double dtc = 0.8 * a / (0.1 + a) * EXP(apx, 0.5 * (Ls - 1.1));
  double flux[8]; /* flux[j]: net X_j -> X_{j+1 mod 8} */
  flux[0] = 1.5 * R[7] * X[0] - 0.1 * X[1];
  for (int j = 1; j <= 6; ++j) flux[j] = 1.0 * X[j] - 0.2 * X[j + 1];
  flux[7] = dtc * X[7] - 1e-4 * X[0];
  for (int j = 0; j < 8; ++j) d[47 + j] = flux[(j + 7) % 8] - flux[j];

  /* I: mechanics */
  const double Fn = 0.25 * X[4] + 0.5 * X[5] + 0.75 * X[6] + X[7];
  d[55] = (1.1 - Ls) / 20.0 - 0.02 * Fn;
  d[56] = (Fn - gam) / 5.0;
}

void or_st57_rhs(double Cm, const double* y, double I, double* d) { st57_rhs(0, Cm, y, I, d); }

/* ST57 with every exp replaced by exp* (eq. apx-e-function) and every log by
 * log* (figure apxlog), as the thesis does for its Shorten model. */
void or_st57_apx_rhs(double Cm, const double* y, double I, double* d) {
  st57_rhs(1, Cm, y, I, d);
}

/* ---------------------------------------------------------------------- */
/* Resting state: damped Newton on G(y) = 0 with the seven conserved sums  */
/* fixed (one equation of each conserving block replaced by its sum).      */
/* ---------------------------------------------------------------------- */

static void rest_residual(int apx, const double* y, double* F) {
  st57_rhs(apx, 1.0, y, 0.0, F);
  double inv[6];
  or_st57_invariants(y, inv);
  F[17] = inv[0] - 1.0;     /* sum P */
  F[38] = inv[1] - 1.0;     /* sum Q */
  F[46] = inv[2] - 1.0;     /* sum R */
  F[54] = inv[3] - 1.0;     /* sum X */
  F[18] = inv[4] - 2200.0;  /* total Ca */
  F[26] = inv[5] - 1500.0;  /* total Mg */
}

/* Gaussian elimination with partial pivoting on an n x n system (in place). */
static int gauss_solve(int nn, double* A, double* b) {
  for (int k = 0; k < nn; ++k) {
    int p = k;
    for (int i = k + 1; i < nn; ++i)
      if (fabs(A[i * nn + k]) > fabs(A[p * nn + k])) p = i;
    if (A[p * nn + k] == 0.0) return -1;
    if (p != k) {
      for (int j = 0; j < nn; ++j) {
        double t = A[k * nn + j];
        A[k * nn + j] = A[p * nn + j];
        A[p * nn + j] = t;
      }
      double t = b[k];
      b[k] = b[p];
      b[p] = t;
    }
    for (int i = k + 1; i < nn; ++i) {
      double f = A[i * nn + k] / A[k * nn + k];
      for (int j = k; j < nn; ++j) A[i * nn + j] -= f * A[k * nn + j];
      b[i] -= f * b[k];
    }
  }
  for (int i = nn - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < nn; ++j) s -= A[i * nn + j] * b[j];
    b[i] = s / A[i * nn + i];
  }
  return 0;
}

/* Initial guess: HH-like resting membranes, uniform chains, Ca buffers at
 * a resting free Ca of 0.1 uM, ions at their targets. */
static void rest_guess(double* y) {
  memset(y, 0, sizeof(double) * ST_N);
  y[0] = -75.0; y[1] = 0.053; y[2] = 0.596; y[3] = 0.318;
  y[4] = -75.0; y[5] = 0.053; y[6] = 0.596; y[7] = 0.318;
  for (int i = 8; i <= 17; ++i) y[i] = 0.1;
  y[18] = 0.1; y[19] = 1500.0; y[20] = 1500.0;
  y[21] = 10.0; y[22] = 100.0; y[23] = 700.0; y[24] = 4.0; y[25] = 400.0; y[26] = 400.0;
  y[27] = 16900.0; y[28] = 16900.0;
  y[29] = 10.0; y[30] = 140.0; y[31] = 5.0; y[32] = 140.0; y[33] = 5.0; y[34] = 128.0;
  for (int i = 35; i <= 38; ++i) y[i] = 0.25;
  for (int i = 39; i <= 46; ++i) y[i] = 0.125;
  for (int i = 47; i <= 54; ++i) y[i] = 0.125;
  y[55] = 1.1; y[56] = 0.0;
}

/* Returns 0 on convergence (max |residual| < 1e-11 after scaling), -1 else;
 * `iters` (nullable) receives the iteration count. */
static int st57_rest(int apx, double* y, int* iters) {
  double F[ST_N], Fp[ST_N], J[ST_N * ST_N], yp[ST_N], dx[ST_N];
  rest_guess(y);
  for (int it = 0; it < 200; ++it) {
    rest_residual(apx, y, F);
    double norm = 0.0;
    for (int i = 0; i < ST_N; ++i) norm = fmax(norm, fabs(F[i]));
    if (iters) *iters = it;
    if (norm < 1e-11) return 0;
    for (int j = 0; j < ST_N; ++j) {
      memcpy(yp, y, sizeof yp);
      double e = 1e-7 * fmax(1.0, fabs(y[j]));
      yp[j] += e;
      rest_residual(apx, yp, Fp);
      for (int i = 0; i < ST_N; ++i) J[i * ST_N + j] = (Fp[i] - F[i]) / e;
    }
    for (int i = 0; i < ST_N; ++i) dx[i] = -F[i];
    if (gauss_solve(ST_N, J, dx)) return -1;
    /* damping: halve the step until the residual does not grow and
       concentrations and probabilities stay positive */
    double lam = 1.0;
    for (int k = 0; k < 40; ++k) {
      int ok = 1;
      for (int i = 0; i < ST_N; ++i) {
        yp[i] = y[i] + lam * dx[i];
        if (i >= 8 && i != 55 && i != 56 && yp[i] < 0.0) ok = 0;
      }
      if (ok) {
        rest_residual(apx, yp, Fp);
        double np = 0.0;
        for (int i = 0; i < ST_N; ++i) np = fmax(np, fabs(Fp[i]));
        if (np < norm || np < 1e-11) break;
      }
      lam *= 0.5;
    }
    memcpy(y, yp, sizeof yp);
  }
  return -1;
}

int or_st57_rest(double* y, int* iters) { return st57_rest(0, y, iters); }
int or_st57_apx_rest(double* y, int* iters) { return st57_rest(1, y, iters); }
