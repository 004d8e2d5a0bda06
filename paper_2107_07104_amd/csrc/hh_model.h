// Hodgkin-Huxley membrane in FP32 for gfx950 (thesis section "Subcellular
// Model", eqs. subcellular_model_helper3-5 and subcellular; rate functions of
// Hodgkin & Huxley 1952 in the -75 mV resting-potential convention of the
// generated-code excerpt in section "Computation of CellML Models").
//
// State (V, m, h, n); V in mV, rates in 1/ms.  With v = V + 75:
//   alpha_m = 0.1 (25-v) / (exp((25-v)/10) - 1)   beta_m = 4 exp(-v/18)
//   alpha_h = 0.07 exp(-v/20)                      beta_h = 1 / (exp((30-v)/10) + 1)
//   alpha_n = 0.01 (10-v) / (exp((10-v)/10) - 1)  beta_n = 0.125 exp(-v/80)
//   I_ion = 120 m^3 h (V - 40) + 36 n^4 (V + 87) + 0.3 (V + 64.387)
//   dV/dt = (I_stim - I_ion) / Cm,  dy/dt = alpha_y (1 - y) - beta_y y.
//
// Every exponential is one v_exp_f32 (2^x) whose argument is a single FMA in
// V: the 1/ln 2 factor, the 1/10, 1/18, 1/20, 1/80 slopes, the +75 shift and
// the prefactors 4, 0.07, 0.125 (as +log2 of the prefactor) are folded into
// the FMA's constants.  The three exponentials of slope -1/10 differ only by
// constant factors, exp(-(V+65)/10) = exp(-(V+50)/10) e^-1.5 and
// exp(-(V+45)/10) = exp(-(V+50)/10) e^0.5, so they take one v_exp_f32 and
// two multiplications.
//
// The APX variant replaces every exponential by exp*(x) = (1 + x/n)^n,
// n = 1024 (eq. apx-e-function).  Ten squarings of 1 + x/n in FP32 would
// multiply the rounding error of 1 + x/n by 1024 (6e-5 relative); instead
// d = exp*(x) - 1 is carried through the ten squarings as d <- d (d + 2),
// starting from d = x/n (one FMA in V), which keeps it to a few ulp and
// gives x / (exp*(x) - 1) = x / d without cancellation.
#pragma once

#include <hip/hip_runtime.h>

namespace fib {
namespace hh {

constexpr double kL2E = 1.4426950408889634074;  // 1 / ln 2

// exp(s * (V + shift)) * pre  ==  2^(V * K1 + K0)
struct ExpCoef {
  float k1, k0;  // 2^(V k1 + k0)
  float a1, a0;  // x / n = V a1 + a0 (exp* variant)
  float pre;     // prefactor (exp* variant)
};
// pre exp(slope (V + shift)), log2_pre = log2(pre)
constexpr ExpCoef exp_coef(double slope, double shift, double pre, double log2_pre) {
  return ExpCoef{(float)(slope * kL2E), (float)(slope * shift * kL2E + log2_pre),
                 (float)(slope / 1024.0), (float)(slope * shift / 1024.0), (float)pre};
}

// log2 of the prefactors
constexpr double kLog2_4 = 2.0;
constexpr double kLog2_007 = -3.8365012677171206;  // log2(0.07)
constexpr double kLog2_0125 = -3.0;

constexpr ExpCoef kBm = exp_coef(-1.0 / 18.0, 75.0, 4.0, kLog2_4);       // 4 exp(-v/18)
constexpr ExpCoef kAh = exp_coef(-1.0 / 20.0, 75.0, 0.07, kLog2_007);    // 0.07 exp(-v/20)
constexpr ExpCoef kBh = exp_coef(-1.0 / 10.0, 45.0, 1.0, 0.0);           // exp((30-v)/10)
constexpr ExpCoef kBn = exp_coef(-1.0 / 80.0, 75.0, 0.125, kLog2_0125);  // 0.125 exp(-v/80)
constexpr ExpCoef kXm = exp_coef(-1.0 / 10.0, 50.0, 1.0, 0.0);  // exp(x_m), x_m = (25-v)/10
constexpr ExpCoef kXn = exp_coef(-1.0 / 10.0, 65.0, 1.0, 0.0);  // exp(x_n), x_n = (10-v)/10

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// exp*(x) - 1 for x / n = V a1 + a0: ten squarings of 1 + x/n in the form
// d <- d (d + 2).
__device__ __forceinline__ float exp_star_m1(float V, const ExpCoef& c) {
  float d = fmaf(V, c.a1, c.a0);
#pragma unroll
  for (int i = 0; i < 10; ++i) d = fmaf(d, d, d + d);
  return d;
}

// c x / (exp(x) - 1) from cx = c x and e = exp(x).  The quotient is 0/0 at
// x = 0, and its cancellation error, about 1.2e-7 / |x| relative, grows as
// x shrinks; for |x| < 4.9e-4 its limit c replaces it, whose error |x|/2 is
// below 2.5e-4 there.  Either way the rate is that inexact only within
// 0.005 mV of the singular voltage.
__device__ __forceinline__ float cx_over_expm1(float cx, float e, float c) {
  const float q = cx * rcp(e - 1.0f);
  return fabsf(cx) < c * 4.9e-4f ? c : q;
}

// Every state is carried as its offset from the resting state (ref): the
// increments of a node near rest are tiny next to the states themselves
// (V ~ -75 mV, h ~ 0.6), and FP32 keeps them only when they are added to
// values near zero.
struct State {
  float V, m, h, n;  // y - ref
};

struct Ref {
  float V, m, h, n;  // resting state
};

// Right-hand side G(y) of the membrane model with stimulus current I
// (APX: with exp* in the rates) at the absolute state (V, m, h, n), with
// the V component scaled by Cm: it returns I - I_ion, the gate components
// are G's own.
template <bool APX = false>
__device__ __forceinline__ State rhs_abs_cm(const State& a, float I) {
  const float V = a.V, m = a.m, h = a.h, n = a.n;
  const float xm = fmaf(V, -0.1f, -5.0f);   // (25 - v)/10 = -(V + 50)/10
  float am, an, bm, ah, bh, bn;
  if constexpr (!APX) {
    constexpr float kEm15 = 0.22313016014842982893f;  // e^-1.5
    constexpr float kE05 = 1.6487212707001281468f;    // e^0.5
    const float xn10 = fmaf(V, -0.01f, -0.65f);       // x_n / 10, x_n = (10 - v)/10
    const float em = ex2(fmaf(V, kXm.k1, kXm.k0));
    const float en = em * kEm15;                      // exp(x_n)
    am = cx_over_expm1(xm, em, 1.0f);
    an = cx_over_expm1(xn10, en, 0.1f);
    bm = ex2(fmaf(V, kBm.k1, kBm.k0));
    ah = ex2(fmaf(V, kAh.k1, kAh.k0));
    bh = rcp(fmaf(em, kE05, 1.0f));                   // 1 / (exp((30-v)/10) + 1)
    bn = ex2(fmaf(V, kBn.k1, kBn.k0));
  } else {
    // x / (exp*(x) - 1) = x / d; near x = 0 its series 1 - (n-1)/(2n) x
    // (truncation below 1e-7 for |x| < 1e-3)
    constexpr float kA = 1023.0f / 2048.0f;
    const float xn = fmaf(V, -0.1f, -6.5f);   // (10 - v)/10 = -(V + 65)/10
    const float dm = exp_star_m1(V, kXm), dn = exp_star_m1(V, kXn);
    am = fabsf(xm) < 1e-3f ? fmaf(xm, -kA, 1.0f) : xm * rcp(dm);
    an = 0.1f * (fabsf(xn) < 1e-3f ? fmaf(xn, -kA, 1.0f) : xn * rcp(dn));
    bm = kBm.pre * (exp_star_m1(V, kBm) + 1.0f);
    ah = kAh.pre * (exp_star_m1(V, kAh) + 1.0f);
    bh = rcp(exp_star_m1(V, kBh) + 2.0f);
    bn = kBn.pre * (exp_star_m1(V, kBn) + 1.0f);
  }

  // I_ion = 120 m^3 h (V - 40) + 36 n^4 (V + 87) + 0.3 (V + 64.387), each
  // driving force with its conductance folded in (one FMA in V each)
  const float m2 = m * m;
  const float m3h = m2 * (m * h);
  const float n2 = n * n;
  const float n4 = n2 * n2;
  const float fna = fmaf(V, 120.0f, -120.0f * 40.0f);
  const float fk = fmaf(V, 36.0f, 36.0f * 87.0f);
  const float fl = fmaf(V, 0.3f, 0.3f * 64.387f);
  const float iion = fmaf(m3h, fna, fmaf(n4, fk, fl));

  State d;
  d.V = I - iion;
  d.m = fmaf(-(am + bm), m, am);
  d.h = fmaf(-(ah + bh), h, ah);
  d.n = fmaf(-(an + bn), n, an);
  return d;
}

__device__ __forceinline__ State absolute(const State& y, const Ref& ref) {
  return State{y.V + ref.V, y.m + ref.m, y.h + ref.h, y.n + ref.n};
}

// G(y) itself, y as offsets from ref: dV/dt = (I - I_ion) / Cm.
template <bool APX = false>
__device__ __forceinline__ State rhs(const State& y, float I, float inv_cm, const Ref& ref) {
  State d = rhs_abs_cm<APX>(absolute(y, ref), I);
  d.V *= inv_cm;
  return d;
}

// One Heun step of width tau (eq. heun):
//   y+ = y + tau/2 (G(y) + G(y + tau G(y))),
// with 1/Cm of the V component folded into its step width.  The stage
// state is formed in absolute values from the first one; the increment is
// added to the offsets.
template <bool APX = false>
__device__ __forceinline__ void heun(State& y, float I, float tau, float inv_cm, const Ref& ref) {
  const float tv = tau * inv_cm;
  const State a1 = absolute(y, ref);
  const State k1 = rhs_abs_cm<APX>(a1, I);
  State a2;
  a2.V = fmaf(tv, k1.V, a1.V);
  a2.m = fmaf(tau, k1.m, a1.m);
  a2.h = fmaf(tau, k1.h, a1.h);
  a2.n = fmaf(tau, k1.n, a1.n);
  const State k2 = rhs_abs_cm<APX>(a2, I);
  const float ht = 0.5f * tau;
  y.V = fmaf(0.5f * tv, k1.V + k2.V, y.V);
  y.m = fmaf(ht, k1.m + k2.m, y.m);
  y.h = fmaf(ht, k1.h + k2.h, y.h);
  y.n = fmaf(ht, k1.n + k2.n, y.n);
}

}  // namespace hh
}  // namespace fib
