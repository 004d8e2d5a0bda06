// ST57, the 57-state Shorten-type stand-in subcellular model, in FP32 for
// gfx950.  Written from the model's specification table (membrane of the
// thesis's section "Subcellular Model" as states 0-3, plus tubular
// compartment, voltage-sensor chain, Ca/Mg buffering, ion concentrations
// with Nernst potentials, Na/K pump cycle, thin-filament chain, cross-bridge
// cycle and mechanics), independently of any other implementation.
//
// States are carried as offsets u = y - ref from the resting state ref (as
// for the Hodgkin-Huxley model); the right-hand side adds ref back.
// Exponentials are 2^x with the slope, shift and 1/ln 2 folded into one
// FMA; logarithms are log2 times ln 2.  The right-hand side is a template:
// the kernels evaluate it in FP32 with v_exp_f32 / v_log_f32 / v_rcp_f32,
// the host evaluates it in FP64 with the C library for the resting-state
// search.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace fib {
namespace st57 {

constexpr int S = 57;
constexpr double kT = 26.71;                     // RT/F, mV
constexpr double kL2E = 1.4426950408889634074;   // 1/ln 2
constexpr double kTln2 = 26.71 * 0.69314718055994530942;

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float lg2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ float fabs_(float x) { return fabsf(x); }
__device__ __forceinline__ float fmax_(float a, float b) { return fmaxf(a, b); }
// FP64 versions for the host's resting-state search (also declared for the
// device so that overload resolution succeeds in both compilation passes).
inline __host__ __device__ double ex2(double x) { return exp2(x); }
inline __host__ __device__ double lg2(double x) { return log2(x); }
inline __host__ __device__ double rcp(double x) { return 1.0 / x; }
inline __host__ __device__ double fma_(double a, double b, double c) { return a * b + c; }
inline __host__ __device__ double fabs_(double x) { return fabs(x); }
inline __host__ __device__ double fmax_(double a, double b) { return a > b ? a : b; }

// c x / (exp(x) - 1) from cx = c x and e = exp(x).  The quotient is 0/0 at
// x = 0, and its cancellation error in FP32, about 1.2e-7 / |x| relative,
// grows as x shrinks; for |x| < 4.9e-4 its limit c replaces it (error
// |x|/2 < 2.5e-4 there, far below FP32 resolution in FP64).
template <typename T>
__host__ __device__ __forceinline__ T cxm1(T cx, T e, T c) {
  return fabs_(cx) < c * T(4.9e-4) ? c : cx * rcp(e - T(1));
}

// ---------------------------------------------------------------------------
// The thesis's approximations (section "Evaluation of Code Generator
// Optimizations"), for the model variant with APX = true.
// ---------------------------------------------------------------------------

// exp*(x) - 1 with exp*(x) = (1 + x/1024)^1024 (eq. apx-e-function): ten
// squarings carried as d <- d (d + 2) from d = x / 1024, so the rounding of
// 1 + x/1024 is not multiplied by 1024.
template <typename T>
__host__ __device__ __forceinline__ T expm1_star(T x) {
  T d = x * T(1.0 / 1024.0);
#pragma unroll
  for (int i = 0; i < 10; ++i) d = fma_(d, d, d + d);
  return d;
}

// c x / (exp*(x) - 1), with its series c (1 - (1023/2048) x) for |x| < 1e-3
// (truncation below 1e-7 relative).
template <typename T>
__host__ __device__ __forceinline__ T cxm1_star(T x, T c) {
  return fabs_(x) < T(1e-3) ? c * fma_(x, T(-1023.0 / 2048.0), T(1))
                            : c * x * rcp(expm1_star(x));
}

// log*(x) (figure apxlog): the argument is scaled by powers of two into
// [0.2, 20), which is exact; the sixth-order Taylor polynomial of log around
// a = 1 (m < 2), 3 (m < 6) or 9 gives y, and one Newton step on
// exp*(y) = m, y - (1 - m / exp*(y)), makes it the inverse of exp*.  The
// scaling loops stop after 160 halvings or doublings (non-finite or zero
// arguments give a non-finite or meaningless result, as log does).
template <typename T>
__host__ __device__ __forceinline__ T log_star(T x) {
  T m = x, k = T(0);
  for (int i = 0; i < 160 && m >= T(20); ++i) {
    m *= T(0.5);
    k += T(1);
  }
  for (int i = 0; i < 160 && m < T(0.2); ++i) {
    m *= T(2);
    k -= T(1);
  }
  const bool p1 = m < T(2), p3 = m < T(6);
  const T inv_a = p1 ? T(1) : (p3 ? T(1.0 / 3.0) : T(1.0 / 9.0));
  const T log_a = p1 ? T(0) : (p3 ? T(1.0986122886681098) : T(2.1972245773362196));
  const T u = fma_(m, inv_a, T(-1));
  // u - u^2/2 + u^3/3 - u^4/4 + u^5/5 - u^6/6 by Horner's rule
  T q = fma_(u, T(-1.0 / 6.0), T(1.0 / 5.0));
  q = fma_(u, q, T(-0.25));
  q = fma_(u, q, T(1.0 / 3.0));
  q = fma_(u, q, T(-0.5));
  q = fma_(u, q, T(1));
  T y = fma_(u, q, log_a);
  y = y - T(1) + m * rcp(expm1_star(y) + T(1));
  return fma_(k, T(0.69314718055994530942), y);
}

// Hodgkin-Huxley gate derivatives at voltage V for gates (m, h, n).  The
// arguments of alpha_m, alpha_n and beta_h have slope -1/10 in V and differ
// by constants: x_n = x_m - 3/2 and beta_h's exponent is x_m + 1/2, so one
// exponential serves the three.  With APX every rate takes its own exp*
// (exp* of a sum is not the product of the exp*s).
template <typename T, bool APX = false>
__host__ __device__ __forceinline__ void hh_gates(T V, T m, T h, T n, T& dm, T& dh, T& dn) {
  T am, an, bm, ah, bh, bn;
  if constexpr (!APX) {
    const T xm = fma_(V, T(-0.1), T(-5.0));        // (25 - v)/10
    const T xn10 = fma_(V, T(-0.01), T(-0.65));    // x_n / 10, x_n = (10 - v)/10
    const T em = ex2(xm * T(kL2E));
    am = cxm1(xm, em, T(1));
    an = cxm1(xn10, em * T(0.22313016014842982893), T(0.1));  // e^-1.5
    // 4 exp(-(V+75)/18), 0.07 exp(-(V+75)/20), 1/(exp(-(V+45)/10)+1), 0.125 exp(-(V+75)/80)
    bm = ex2(fma_(V, T(-kL2E / 18.0), T(-75.0 * kL2E / 18.0 + 2.0)));
    ah = ex2(fma_(V, T(-kL2E / 20.0), T(-75.0 * kL2E / 20.0 - 3.8365012677171206)));
    bh = rcp(fma_(em, T(1.6487212707001281468), T(1)));  // e^0.5
    bn = ex2(fma_(V, T(-kL2E / 80.0), T(-75.0 * kL2E / 80.0 - 3.0)));
  } else {
    am = cxm1_star(fma_(V, T(-0.1), T(-5.0)), T(1));    // x_m = -(V + 50)/10
    an = cxm1_star(fma_(V, T(-0.1), T(-6.5)), T(0.1));  // x_n = -(V + 65)/10
    bm = T(4) * (expm1_star(fma_(V, T(-1.0 / 18.0), T(-75.0 / 18.0))) + T(1));
    ah = T(0.07) * (expm1_star(fma_(V, T(-1.0 / 20.0), T(-75.0 / 20.0))) + T(1));
    bh = rcp(expm1_star(fma_(V, T(-0.1), T(-4.5))) + T(2));
    bn = T(0.125) * (expm1_star(fma_(V, T(-1.0 / 80.0), T(-75.0 / 80.0))) + T(1));
  }
  dm = fma_(-(am + bm), m, am);
  dh = fma_(-(ah + bh), h, ah);
  dn = fma_(-(an + bn), n, an);
}

// Right-hand side at absolute states y: d = G(y) with stimulus current I
// (uA/cm^2).  APX: every exp replaced by exp* and every log by log*, applied
// to the arguments as the model writes them (the Nernst ratios).
template <typename T, bool APX = false>
__host__ __device__ __forceinline__ void rhs_abs(const T (&y)[S], T I, T inv_cm, T (&d)[S]) {
  using F = T;

  const F V = y[0], m = y[1], h = y[2], n = y[3];
  const F Vt = y[4], mt = y[5], ht = y[6], nt = y[7];
  const F cm = y[18], cs = y[19], cj = y[20], bT = y[21], bP = y[22], gP = y[23],
              bA = y[24], gA = y[25], gm = y[26], bC = y[27], bCj = y[28];
  const F Nai = y[29], Ki = y[30], Cli = y[31], Nat = y[32], Kt = y[33], Clt = y[34];

  // Na/K pump cycle (states 35-38)
  const F na3 = Nai * Nai * Nai;
  const F k1 = na3 * rcp(F(1000.0) + na3);
  F k2;
  if constexpr (!APX)
    k2 = F(0.8) * ex2(V * F(0.3 * kL2E / kT));
  else
    k2 = F(0.8) * (expm1_star(V * F(0.3 / kT)) + F(1));
  const F kt2 = Kt * Kt;
  const F k3 = F(1.2) * kt2 * rcp(F(2.25) + kt2);
  const F J01 = fma_(k1, y[35], -F(0.05) * y[36]);
  const F J12 = fma_(k2, y[36], -F(0.05) * y[37]);
  const F J23 = fma_(k3, y[37], -F(0.02) * y[38]);
  const F J30 = fma_(F(0.6), y[38], -F(0.01) * y[35]);
  d[35] = J30 - J01;
  d[36] = J01 - J12;
  d[37] = J12 - J23;
  d[38] = J23 - J30;
  const F Jp = J12;

  // surface membrane (states 0-3)
  const F m3h = m * m * m * h;
  const F n4 = (n * n) * (n * n);
  const F INas = F(120.0) * m3h * (V - F(40.0));
  const F IKs = F(36.0) * n4 * (V + F(87.0));
  const F ILs = F(0.3) * (V + F(64.387));
  // E_Cl = -kT ln(128 / Cl_i) = kT ln 2 (log2 Cl_i - 7)
  F ECl;
  if constexpr (!APX)
    ECl = F(kTln2) * (lg2(Cli) - F(7.0));
  else
    ECl = F(-kT) * log_star(F(128.0) * rcp(Cli));
  const F IClS = F(0.05) * (V - ECl);
  const F Ic = F(0.2) * (V - Vt);
  d[0] = (I - (INas + IKs + ILs) - IClS - Ic - F(0.2) * Jp) * inv_cm;
  hh_gates<T, APX>(V, m, h, n, d[1], d[2], d[3]);

  // tubular membrane (states 4-7), Nernst potentials from concentrations
  F ENa, EK, EClt;
  if constexpr (!APX) {
    const F lNai = lg2(Nai), lKi = lg2(Ki), lCli = lg2(Cli);
    ENa = F(kTln2) * (lg2(Nat) - lNai);
    EK = F(kTln2) * (lg2(Kt) - lKi);
    EClt = F(-kTln2) * (lg2(Clt) - lCli);
  } else {
    ENa = F(kT) * log_star(Nat * rcp(Nai));
    EK = F(kT) * log_star(Kt * rcp(Ki));
    EClt = F(-kT) * log_star(Clt * rcp(Cli));
  }
  const F INat = F(12.0) * (mt * mt * mt * ht) * (Vt - ENa);
  const F IKt = F(3.6) * ((nt * nt) * (nt * nt)) * (Vt - EK);
  const F IClt = F(0.05) * (Vt - EClt);
  d[4] = (F(0.8) * (V - Vt) - (INat + IKt + IClt + F(0.1) * Jp)) * inv_cm;
  hh_gates<T, APX>(Vt, mt, ht, nt, d[5], d[6], d[7]);

  // voltage-sensor chain (states 8-17): rates exp(+-(Vt - V_i)/25),
  // V_i = -70 + 7.5 i, as E exp(-V_i/25) and exp(V_i/25) / E with
  // E = exp(Vt/25): one exponential and one reciprocal for the eighteen
  {
    // exp(-V_i/25) and exp(V_i/25)
    constexpr double kCf[9] = {16.444646771097048, 12.182493960703473, 9.025013499434122, 6.6858944422792685, 4.953032424395115, 3.6692966676192444, 2.718281828459045, 2.0137527074704766, 1.4918246976412703};
    constexpr double kCb[9] = {0.06081006262521797, 0.0820849986238988, 0.11080315836233387, 0.14956861922263506, 0.20189651799465538, 0.2725317930340126, 0.36787944117144233, 0.4965853037914095, 0.6703200460356393};
    F kf[9], kb[9];
    if constexpr (!APX) {
      const F E = ex2(Vt * F(kL2E / 25.0));
      const F Einv = rcp(E);
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        kf[i] = E * F(kCf[i]);
        kb[i] = Einv * F(kCb[i]);
      }
    } else {
      // exp*((V_t - V_i)/25) and exp*(-(V_t - V_i)/25), V_i = -70 + 7.5 i
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const F x = fma_(Vt, F(1.0 / 25.0), F((70.0 - 7.5 * i) / 25.0));
        kf[i] = expm1_star(x) + F(1);
        kb[i] = expm1_star(-x) + F(1);
      }
    }
    F flow[9];  // net P_i -> P_{i+1}
#pragma unroll
    for (int i = 0; i < 9; ++i) flow[i] = fma_(kf[i], y[8 + i], -kb[i] * y[9 + i]);
    d[8] = -flow[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) d[8 + i] = flow[i - 1] - flow[i];
    d[17] = flow[8];
  }

  // calcium and magnesium (states 18-28)
  const F P9 = y[17];
  const F fload = cj > F(500.0) ? F(1.0) : cj * (F(1.0) / F(500.0));
  const F Jrel = P9 * fload * (cj - cm);
  const F Jleak = F(2e-5) * (cj - cm);
  const F cp = fmax_(cm, F(0.0));
  const F cp2 = cp * cp;
  const F Jup = F(4.0) * cp2 * rcp(F(1.0) + cp2);
  const F Jtr = F(0.02) * (cs - cj);
  const F RT = fma_(F(0.0885) * cm, F(140.0) - bT, -F(0.115) * bT);
  const F freeP = F(1500.0) - bP - gP;
  const F RP = fma_(F(0.0417) * cm, freeP, -F(5e-4) * bP);
  const F RPM = fma_(F(3.3e-5) * gm, freeP, -F(3e-3) * gP);
  const F freeA = F(8000.0) - bA - gA;
  const F RA = fma_(F(0.15) * cm, freeA, -F(30.0) * bA);
  const F RAM = fma_(F(1.5e-3) * gm, freeA, -F(0.15) * gA);
  const F RC = fma_(F(4e-4) * cs, F(31000.0) - bC, -F(0.5) * bC);
  const F RCj = fma_(F(4e-4) * cj, F(31000.0) - bCj, -F(0.5) * bCj);
  d[18] = Jrel + Jleak - Jup - RT - RP - RA;
  d[19] = (Jup - Jtr) * F(10.0) - RC;
  d[20] = (Jtr - Jrel - Jleak) * F(100.0) - RCj;
  d[21] = RT;
  d[22] = RP;
  d[23] = RPM;
  d[24] = RA;
  d[25] = RAM;
  d[26] = -(RPM + RAM);
  d[27] = RC;
  d[28] = RCj;

  // ion concentrations (states 29-34)
  const F Ip = F(0.6) * Jp;  // 0.2 Jp (surface) + 4 * 0.1 Jp (tubule)
  d[29] = fma_(-F(2e-5), INas + F(4.0) * INat + F(3.0) * Ip, -(Nai - F(10.0)) * F(1e-3));
  d[30] = fma_(-F(2e-5), IKs + F(4.0) * IKt - F(2.0) * Ip, -(Ki - F(140.0)) * F(1e-3));
  d[31] = fma_(F(2e-5), IClS + F(4.0) * IClt, -(Cli - F(5.0)) * F(1e-3));
  d[32] = fma_(F(2e-3), INat + F(0.3) * Jp, -(Nat - F(140.0)) * F(0.02));
  d[33] = fma_(F(2e-3), IKt - F(0.2) * Jp, -(Kt - F(5.0)) * F(0.02));
  d[34] = fma_(-F(2e-3), IClt, -(Clt - F(128.0)) * F(0.02));

  // thin-filament chain (states 39-46)
  {
    const F th = bT * (F(1.0) / F(140.0));
    const F rf = fma_(F(2.0) * th, th, F(1e-3));
    const F rb = F(0.3) * rcp(fma_(F(5.0), th, F(1.0)));
    F flow[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) flow[i] = fma_(rf, y[39 + i], -rb * y[40 + i]);
    d[39] = -flow[0];
#pragma unroll
    for (int i = 1; i < 7; ++i) d[39 + i] = flow[i - 1] - flow[i];
    d[46] = flow[6];
  }

  // cross-bridge cycle (states 47-54) and mechanics (55-56)
  {
    const F a = gA * (F(1.0) / F(8000.0));
    const F Ls = y[55];
    F ed;
    if constexpr (!APX)
      ed = ex2(fma_(Ls, F(0.5 * kL2E), F(-0.55 * kL2E)));
    else
      ed = expm1_star(fma_(Ls, F(0.5), F(-0.55))) + F(1);
    const F det = F(0.8) * a * rcp(F(0.1) + a) * ed;
    F flux[8];
    flux[0] = fma_(F(1.5) * y[46], y[47], -F(0.1) * y[48]);
#pragma unroll
    for (int j = 1; j <= 6; ++j) flux[j] = fma_(-F(0.2), y[48 + j], y[47 + j]);
    flux[7] = fma_(det, y[54], -F(1e-4) * y[47]);
    d[47] = flux[7] - flux[0];
#pragma unroll
    for (int j = 1; j < 8; ++j) d[47 + j] = flux[j - 1] - flux[j];
    const F Fn = fma_(F(0.25), y[51], fma_(F(0.5), y[52], fma_(F(0.75), y[53], y[54])));
    d[55] = fma_(F(1.1) - Ls, F(0.05), -F(0.02) * Fn);
    d[56] = (Fn - y[56]) * F(0.2);
  }
}

// Right-hand side at offsets: d = G(ref + u).  `ref` points at S values
// (kernel arguments, uniform across lanes).
template <typename T, bool APX = false>
__host__ __device__ __forceinline__ void rhs(const T (&u)[S], const T* __restrict__ ref, T I,
                                             T inv_cm, T (&d)[S]) {
  T y[S];
#pragma unroll
  for (int k = 0; k < S; ++k) y[k] = u[k] + ref[k];
  rhs_abs<T, APX>(y, I, inv_cm, d);
}

// One Heun step of width tau on the offsets u (eq. heun).  The update is
// arranged so that only two 57-vectors are live while the second stage
// is evaluated.
template <bool APX = false>
__device__ __forceinline__ void heun(float (&u)[S], const float* __restrict__ ref, float I,
                                     float tau, float inv_cm) {
  float k[S];
  rhs<float, APX>(u, ref, I, inv_cm, k);
  const float ht = 0.5f * tau;
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const float w = fmaf(ht, k[q], u[q]);  // u + tau/2 k1
    k[q] = fmaf(tau, k[q], u[q]);          // stage point u + tau k1
    u[q] = w;
  }
  float k2[S];
  rhs<float, APX>(k, ref, I, inv_cm, k2);
#pragma unroll
  for (int q = 0; q < S; ++q) u[q] = fmaf(ht, k2[q], u[q]);
}

}  // namespace st57
}  // namespace fib
