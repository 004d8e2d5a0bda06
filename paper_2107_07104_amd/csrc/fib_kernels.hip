// HIP kernels of the fiber monodomain solver (gfx950).
//
// Data layout in HBM: structure of arrays, state k of global node i at
// state[k * n_total + i], fibers concatenated in the caller's order.  Row k
// holds state k as its offset y_k - rest_k from the resting state: a node
// near rest (the foot of a propagating front, the quiet part of a fiber)
// takes increments far below the FP32 resolution of -75 mV or of a gate at
// 0.6, and they survive only when added to values near zero.  Without the
// offsets, FP32 rounding of the gates shifts the arrival of a front by about
// a split step over 20 ms; with them the FP32 path tracks the FP64 method to
// a few 1e-7 ms.  The offsets also make checkpoints round-trip exactly.
//
// Work decomposition of the fused and diffusion kernels: fibers are packed
// into "bins" (one workgroup each) of at most threads * K nodes; thread t of
// a bin owns the K consecutive slots t*K .. t*K+K-1 of the bin's
// concatenated fibers.  Fiber boundaries inside a bin are rows without
// coupling, so a bin's Crank-Nicolson matrix is one block-diagonal
// tridiagonal system (eq. discretized_fibers_1) that the partitioned solve
// below handles as a whole.
//
// Partitioned tridiagonal solve (exact up to rounding, see cn_setup /
// cn_solve): in each thread's segment the last slot is an interface unknown
// z_t and the K-1 interior unknowns are eliminated locally, leaving one
// tridiagonal equation per thread in (z_{t-1}, z_t, z_{t+1}); that reduced
// system is solved by parallel cyclic reduction (PCR) through LDS, and the
// interior values follow by back substitution.  The matrix does not change
// between steps, so all elimination factors and PCR multipliers are
// computed once per launch; a step only moves right-hand sides.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "fib_internal.h"
#include "hh_model.h"
#include "st57_model.h"

namespace fib {

// ---------------------------------------------------------------------------
// Lumped Crank-Nicolson rows
// ---------------------------------------------------------------------------

// Row of (dt/2) c M_L^{-1} K for a slot: weights of the left and right
// neighbours.  Linear elements with lumped mass h (1/2, 1, ..., 1, 1/2)
// give (r/2, -r, r/2) inside a fiber and (0, -r, r) / (r, -r, 0) at its
// no-flux ends, r = c dt / h^2.
__device__ __forceinline__ void row_weights(uint32_t info, float r, float& wl, float& wr) {
  const bool L = (info & SLOT_L) != 0u;
  const bool R = (info & SLOT_R) != 0u;
  wl = L ? (R ? 0.5f * r : r) : 0.0f;
  wr = R ? (L ? 0.5f * r : r) : 0.0f;
}

// Coupling bits of a thread's K slots packed two per slot (bits 2q, 2q+1:
// SLOT_L, SLOT_R of slot q), so that they take one register.
template <int K>
__device__ __forceinline__ uint32_t pack_lr(const uint32_t (&info)[K]) {
  uint32_t lr = 0u;
#pragma unroll
  for (int q = 0; q < K; ++q) lr |= (info[q] & (SLOT_L | SLOT_R)) << (2 * q);
  return lr;
}

// LDS layout (floats, T = threads):
//   [0, T)        V of each thread's first slot
//   [T, 2T)       V of each thread's last slot
//   [2T, 3T)      first interior value of y (local solve)
//   [3T, 5T)      PCR right-hand sides, ping-pong
//   [5T, 6T)      interface values z
//   [6T, 6T+2LT)  PCR multipliers alpha_l, gamma_l
template <int K>
struct CNConst {
  float inv[K - 1];   // 1 / pivot of the interior elimination
  float ainv[K - 1];  // a_q / pivot_q
  float cp[K - 1];    // c_q / pivot_q
  float v[K - 1];     // interior response to z_{t-1}
  float w[K - 1];     // interior response to z_t
  float ae, ce;       // couplings of the interface row
  float inv_rd;       // 1 / diagonal of the reduced row after the PCR levels
};

// Elimination factors, interior responses and PCR multipliers for the
// current bin.  Must be called by all threads of the workgroup.  The
// reciprocals are the hardware's (v_rcp_f32, within 1 ulp): the matrix is
// strictly diagonally dominant, so a pivot off by an ulp changes the
// solution by a few ulps, as any rounding of the elimination does.
template <int K>
__device__ void cn_setup(CNConst<K>& cc, uint32_t lr, float r, float* lds, int T, int t,
                         int levels) {
  float a[K], c[K], d[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    float wl, wr;
    row_weights(lr >> (2 * q), r, wl, wr);
    a[q] = -wl;
    c[q] = -wr;
    d[q] = 1.0f + wl + wr;
  }
  // forward elimination over the interior slots 0..K-2 (no pivoting: the
  // matrix is strictly diagonally dominant)
  float vp[K - 1];
#pragma unroll
  for (int q = 0; q < K - 1; ++q) {
    const float den = (q == 0) ? d[0] : fmaf(-a[q], cc.cp[q - 1 < 0 ? 0 : q - 1], d[q]);
    cc.inv[q] = __builtin_amdgcn_rcpf(den);
    cc.ainv[q] = a[q] * cc.inv[q];
    cc.cp[q] = c[q] * cc.inv[q];
    vp[q] = (q == 0) ? -a[0] * cc.inv[0] : -cc.ainv[q] * vp[q - 1 < 0 ? 0 : q - 1];
  }
  // back substitution for the responses to z_{t-1} (v) and z_t (w)
  cc.v[K - 2] = vp[K - 2];
  cc.w[K - 2] = cc.cp[K - 2] * -1.0f;
#pragma unroll
  for (int q = K - 3; q >= 0; --q) {
    cc.v[q] = fmaf(-cc.cp[q], cc.v[q + 1], vp[q]);
    cc.w[q] = -cc.cp[q] * cc.w[q + 1];
  }
  cc.ae = a[K - 1];
  cc.ce = c[K - 1];

  // reduced row of thread t: Ra z_{t-1} + Rd z_t + Rc z_{t+1} = Rb
  float* s_v0 = lds;       // v[0] of each thread
  float* s_w0 = lds + T;   // w[0] of each thread
  s_v0[t] = cc.v[0];
  s_w0[t] = cc.w[0];
  __syncthreads();
  const float vn = (t + 1 < T) ? s_v0[t + 1] : 0.0f;
  const float wn = (t + 1 < T) ? s_w0[t + 1] : 0.0f;
  __syncthreads();
  float Ra = cc.ae * cc.v[K - 2];
  float Rd = d[K - 1] + cc.ae * cc.w[K - 2] + cc.ce * vn;
  float Rc = cc.ce * wn;

  // PCR on the coefficients, once; level l pairs rows t - 2^l and t + 2^l
  float* s_ra = lds;
  float* s_rd = lds + T;
  float* s_rc = lds + 2 * T;
  float* s_al = lds + 6 * T;
  float* s_ga = s_al + levels * T;
  for (int l = 0; l < levels; ++l) {
    const int s = 1 << l;
    s_ra[t] = Ra;
    s_rd[t] = Rd;
    s_rc[t] = Rc;
    __syncthreads();
    const bool hl = t - s >= 0, hr = t + s < T;
    const float ra_l = hl ? s_ra[t - s] : 0.0f, rd_l = hl ? s_rd[t - s] : 1.0f,
                rc_l = hl ? s_rc[t - s] : 0.0f;
    const float ra_r = hr ? s_ra[t + s] : 0.0f, rd_r = hr ? s_rd[t + s] : 1.0f,
                rc_r = hr ? s_rc[t + s] : 0.0f;
    __syncthreads();
    const float al = -Ra * __builtin_amdgcn_rcpf(rd_l);
    const float ga = -Rc * __builtin_amdgcn_rcpf(rd_r);
    s_al[l * T + t] = al;
    s_ga[l * T + t] = ga;
    Rd = Rd + al * rc_l + ga * ra_r;
    Ra = al * ra_l;
    Rc = ga * rc_r;
  }
  cc.inv_rd = __builtin_amdgcn_rcpf(Rd);
  __syncthreads();
}

// One Crank-Nicolson substep on the thread's K slots of V (in registers),
//   (I - dt/2 L) V+ = (I + dt/2 L) V,  L = c M_L^{-1} K,
// for the whole bin.  V may hold V_m or V_m minus any constant (the step
// commutes with adding a constant).  All threads of the workgroup must call
// it.  Bit q of `live` clear zeroes slot q's right-hand side: a fiber whose
// slots are all cleared keeps its V exactly (the matrix is block diagonal
// per fiber and every coupling across a fiber end is an exact zero).
template <int K>
__device__ __forceinline__ void cn_solve(float (&V)[K], uint32_t lr, float r,
                                         float rhs, const CNConst<K>& cc, float* lds, int T,
                                         int t, int levels, uint32_t live) {
  float* s_vf = lds;
  float* s_vl = lds + T;
  float* s_y0 = lds + 2 * T;
  float* s_rb = lds + 3 * T;
  float* s_z = lds + 5 * T;
  const float* s_al = lds + 6 * T;
  const float* s_ga = s_al + levels * T;

  // Increment form: with A = I - theta dt L the step
  // V+ = A^{-1} (I + (1 - theta) dt L) V equals V + d where A d = dt L V
  // (cc holds the factors of A, whose row weights `r` also give dt L: times
  // rhs = 1 / theta).  The right-hand side is built from
  // neighbour differences, so a constant field gives d = 0 exactly and the
  // rounding error of the solve scales with the increment, not with |V|.
  s_vf[t] = V[0];
  s_vl[t] = V[K - 1];
  __syncthreads();
  const float vleft = (t > 0) ? s_vl[t - 1] : 0.0f;
  const float vright = (t + 1 < T) ? s_vf[t + 1] : 0.0f;
  float b[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const float l = (q == 0) ? vleft : V[q == 0 ? 0 : q - 1];
    const float rr = (q == K - 1) ? vright : V[q == K - 1 ? K - 1 : q + 1];
    float wl, wr;
    row_weights(lr >> (2 * q), r, wl, wr);
    // dt L V = (wl (V_l - V) + wr (V_r - V)) / theta with the matrix's
    // weights (theta dt L); a zero weight removes the (possibly unrelated)
    // neighbour value exactly
    b[q] = rhs * fmaf(wl, l - V[q], wr * (rr - V[q]));
    if (!((live >> q) & 1u)) b[q] = 0.0f;
  }
  // interior solve with the right-hand side only
  float y[K - 1];
  y[0] = b[0] * cc.inv[0];
#pragma unroll
  for (int q = 1; q < K - 1; ++q) y[q] = fmaf(-cc.ainv[q], y[q - 1], b[q] * cc.inv[q]);
#pragma unroll
  for (int q = K - 3; q >= 0; --q) y[q] = fmaf(-cc.cp[q], y[q + 1], y[q]);

  // reduced right-hand side needs the next thread's first interior value
  s_y0[t] = y[0];
  __syncthreads();
  const float yn = (t + 1 < T) ? s_y0[t + 1] : 0.0f;
  float rb = fmaf(-cc.ae, y[K - 2], fmaf(-cc.ce, yn, b[K - 1]));

  for (int l = 0; l < levels; ++l) {
    const int s = 1 << l;
    float* buf = s_rb + (l & 1) * T;
    buf[t] = rb;
    __syncthreads();
    const float rl = (t - s >= 0) ? buf[t - s] : 0.0f;
    const float rr = (t + s < T) ? buf[t + s] : 0.0f;
    rb = fmaf(s_al[l * T + t], rl, fmaf(s_ga[l * T + t], rr, rb));
  }
  const float z = rb * cc.inv_rd;

  s_z[t] = z;
  __syncthreads();
  const float zl = (t > 0) ? s_z[t - 1] : 0.0f;
#pragma unroll
  for (int q = 0; q < K - 1; ++q) V[q] += fmaf(cc.v[q], zl, fmaf(cc.w[q], z, y[q]));
  V[K - 1] += z;
}

// One Crank-Nicolson substep with the elimination factors formed on the way,
// for launches with a single substep: the arithmetic of cn_setup followed by
// one cn_solve, operation for operation, with the exchanges of the two
// merged, so a bin needs 3 + L barriers instead of 8 + 2L.  vl and vr are
// the values of the slots left of the thread's first and right of its last
// (0 at the bin's ends, where the weights are zero); X3 (3T floats), P (8T,
// two buffers of four coefficients per thread, alternating by PCR level)
// and Z (T) are LDS arrays that nothing else uses during the call.
template <int K>
__device__ __forceinline__ void cn_merged(float (&V)[K], float vl, float vr, uint32_t lr,
                                          float r, float rhs, uint32_t live, float* X3,
                                          float* P, float* Z, int T, int t, int levels) {
  float a[K], c[K], d[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    float wl, wr;
    row_weights(lr >> (2 * q), r, wl, wr);
    a[q] = -wl;
    c[q] = -wr;
    d[q] = 1.0f + wl + wr;
  }
  float inv[K - 1], ainv[K - 1], cp[K - 1], v[K - 1], w[K - 1];
#pragma unroll
  for (int q = 0; q < K - 1; ++q) {
    const float den = (q == 0) ? d[0] : fmaf(-a[q], cp[q - 1 < 0 ? 0 : q - 1], d[q]);
    inv[q] = __builtin_amdgcn_rcpf(den);
    ainv[q] = a[q] * inv[q];
    cp[q] = c[q] * inv[q];
    v[q] = (q == 0) ? -a[0] * inv[0] : -ainv[q] * v[q - 1 < 0 ? 0 : q - 1];
  }
  w[K - 2] = cp[K - 2] * -1.0f;
#pragma unroll
  for (int q = K - 3; q >= 0; --q) {
    v[q] = fmaf(-cp[q], v[q + 1], v[q]);
    w[q] = -cp[q] * w[q + 1];
  }
  // right-hand side dt L V in increment form and the interior solve
  float b[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const float l = (q == 0) ? vl : V[q == 0 ? 0 : q - 1];
    const float rr = (q == K - 1) ? vr : V[q == K - 1 ? K - 1 : q + 1];
    float wl, wr;
    row_weights(lr >> (2 * q), r, wl, wr);
    b[q] = rhs * fmaf(wl, l - V[q], wr * (rr - V[q]));
    if (!((live >> q) & 1u)) b[q] = 0.0f;
  }
  float y[K - 1];
  y[0] = b[0] * inv[0];
#pragma unroll
  for (int q = 1; q < K - 1; ++q) y[q] = fmaf(-ainv[q], y[q - 1], b[q] * inv[q]);
#pragma unroll
  for (int q = K - 3; q >= 0; --q) y[q] = fmaf(-cp[q], y[q + 1], y[q]);
  // the next thread's responses and interior value give the reduced row
  X3[t] = v[0];
  X3[T + t] = w[0];
  X3[2 * T + t] = y[0];
  __syncthreads();
  const float vn = (t + 1 < T) ? X3[t + 1] : 0.0f;
  const float wn = (t + 1 < T) ? X3[T + t + 1] : 0.0f;
  const float yn = (t + 1 < T) ? X3[2 * T + t + 1] : 0.0f;
  const float ae = a[K - 1], ce = c[K - 1];
  float Ra = ae * v[K - 2];
  float Rd = d[K - 1] + ae * w[K - 2] + ce * vn;
  float Rc = ce * wn;
  float rb = fmaf(-ae, y[K - 2], fmaf(-ce, yn, b[K - 1]));
  for (int l = 0; l < levels; ++l) {
    const int sh = 1 << l;
    float* buf = P + (l & 1) * 4 * T;
    buf[t] = Ra;
    buf[T + t] = Rd;
    buf[2 * T + t] = Rc;
    buf[3 * T + t] = rb;
    __syncthreads();
    const bool hl = t - sh >= 0, hr = t + sh < T;
    const float ra_l = hl ? buf[t - sh] : 0.0f, rd_l = hl ? buf[T + t - sh] : 1.0f,
                rc_l = hl ? buf[2 * T + t - sh] : 0.0f, rb_l = hl ? buf[3 * T + t - sh] : 0.0f;
    const float ra_r = hr ? buf[t + sh] : 0.0f, rd_r = hr ? buf[T + t + sh] : 1.0f,
                rc_r = hr ? buf[2 * T + t + sh] : 0.0f, rb_r = hr ? buf[3 * T + t + sh] : 0.0f;
    const float al = -Ra * __builtin_amdgcn_rcpf(rd_l);
    const float ga = -Rc * __builtin_amdgcn_rcpf(rd_r);
    Rd = Rd + al * rc_l + ga * ra_r;
    Ra = al * ra_l;
    Rc = ga * rc_r;
    rb = fmaf(al, rb_l, fmaf(ga, rb_r, rb));
  }
  const float z = rb * __builtin_amdgcn_rcpf(Rd);
  Z[t] = z;
  __syncthreads();
  const float zl = (t > 0) ? Z[t - 1] : 0.0f;
#pragma unroll
  for (int q = 0; q < K - 1; ++q) V[q] += fmaf(v[q], zl, fmaf(w[q], z, y[q]));
  V[K - 1] += z;
}

// ---------------------------------------------------------------------------
// Fused persistent kernel, Hodgkin-Huxley
// ---------------------------------------------------------------------------

// One workgroup per bin runs split steps step0 .. step0+n_steps-1 with every
// node's four states in registers: V_m prescriptions of the step, R(dt/2)
// D(dt) R(dt/2) (Godunov: R(dt) D(dt), n_sub2 = 0), then the observables.  Device memory is read at the start, written at the end and
// for samples / activation times only.
// APX: the membrane with exp* in its rates (model FIB_MODEL_HH_APX_EXP).
template <int K, int MAXT, bool APX>
__global__ __launch_bounds__(MAXT) void k_run_hh(KArgs A) {
  extern __shared__ float lds[];
  const int T = blockDim.x;
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * A.cap + (int64_t)t * K;
  const int64_t nt = A.n_total;

  uint32_t info[K];
  hh::State y[K];
  uint32_t done = 0;  // bit q: slot q needs no activation-time update
#pragma unroll
  for (int q = 0; q < K; ++q) {
    info[q] = A.slot_info[base + q];
    const int32_t g = A.slot_gidx[base + q];
    if (g >= 0) {
      y[q].V = A.state[g];
      y[q].m = A.state[nt + g];
      y[q].h = A.state[2 * nt + g];
      y[q].n = A.state[3 * nt + g];
      if (!isinf(A.t_act[g])) done |= 1u << q;
    } else {
      y[q] = hh::State{0.0f, 0.0f, 0.0f, 0.0f};
      done |= 1u << q;
    }
  }
  CNConst<K> cc;
  cn_setup<K>(cc, pack_lr<K>(info), A.r_mat, lds, T, t, A.pcr_levels);
  const hh::Ref ref{A.rest[0], A.rest[1], A.rest[2], A.rest[3]};

  const uint32_t all = (K >= 32) ? 0xffffffffu : ((1u << K) - 1u);
  const int32_t n_end = A.step0 + A.n_steps;
  for (int32_t n = A.step0; n < n_end; ++n) {
    float I[K], v0[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
      v0[q] = y[q].V;
      float vp;
      if (stim_eval(info[q] >> SLOT_STIM_SHIFT, A.stim, n, I[q], vp)) y[q].V = vp;
    }
    for (int s = 0; s < A.n_sub; ++s) {
#pragma unroll
      for (int q = 0; q < K; ++q) hh::heun<APX>(y[q], I[q], A.tau, A.inv_cm, ref);
    }
    {
      float V[K];
#pragma unroll
      for (int q = 0; q < K; ++q) V[q] = y[q].V;
      for (int c = 0; c < A.n_cn; ++c)
        cn_solve<K>(V, pack_lr<K>(info), A.r_mat, A.rhs, cc, lds, T, t, A.pcr_levels, ~0u);
#pragma unroll
      for (int q = 0; q < K; ++q) y[q].V = V[q];
    }
    for (int s = 0; s < A.n_sub2; ++s) {
#pragma unroll
      for (int q = 0; q < K; ++q) hh::heun<APX>(y[q], I[q], A.tau, A.inv_cm, ref);
    }
    // activation times: first upward crossing of v_th between step ends
    // (the voltage offsets cross v_th - rest_V)
    if (done != all) {
      const float t0 = (float)n * A.dt;
      const float uth = A.v_th - A.rest[0];
#pragma unroll
      for (int q = 0; q < K; ++q) {
        if (!((done >> q) & 1u) && v0[q] < uth && y[q].V >= uth) {
          const int32_t g = A.slot_gidx[base + q];
          A.t_act[g] = fmaf(A.dt, (uth - v0[q]) / (y[q].V - v0[q]), t0);
          done |= 1u << q;
        }
      }
    }
    if (A.sample_every > 0 && ((int64_t)n + 1) % A.sample_every == 0) {
      const int64_t row = ((int64_t)n + 1) / A.sample_every - 1 - A.sample_row0;
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const int32_t g = A.slot_gidx[base + q];
        if (g >= 0) A.samples[row * nt + g] = y[q].V + A.rest[0];
      }
    }
  }

  bool bad = false;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int32_t g = A.slot_gidx[base + q];
    if (g >= 0) {
      A.state[g] = y[q].V;
      A.state[nt + g] = y[q].m;
      A.state[2 * nt + g] = y[q].h;
      A.state[3 * nt + g] = y[q].n;
      bad |= !isfinite(y[q].V) || !isfinite(y[q].m) || !isfinite(y[q].h) || !isfinite(y[q].n);
    }
  }
  if (bad) atomicOr(A.flag, 1);
}

// ---------------------------------------------------------------------------
// Fused persistent kernel with adaptive computation (Hodgkin-Huxley)
// ---------------------------------------------------------------------------

// Equilibrium check: the relative change |y_k+ - y_k| > tol |y_k| of any
// state over the reaction part (y = offset + rest).
// The same test against the state before the reaction part, read again from
// memory (node i's entry `col` of state row 0, rows `stride` apart) rather
// than held in registers through the substeps.
template <int S>
__device__ __forceinline__ bool state_moved(const float (&u)[S], const float* col, int64_t stride,
                                            const float* rest, float tol) {
  // a new read, not the registers of the first one; typed global so that
  // the loads do not compile to flat instructions
  gfloat* g = (gfloat*)const_cast<float*>(col);
  __asm__("" : "+v"(g));
  bool m = false;
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const float b = g[k * stride];
    m |= fabsf(u[k] - b) > tol * fabsf(b + rest[k]);
  }
  return m;
}

template <int S>
__device__ __forceinline__ bool point_moved(const float (&u)[S], const float (&b)[S],
                                            const float* rest, float tol) {
  bool m = false;
#pragma unroll
  for (int k = 0; k < S; ++k) m |= fabsf(u[k] - b[k]) > tol * fabsf(b[k] + rest[k]);
  return m;
}



// The same split steps as k_run_hh with the adaptive computation of the
// reaction: the bin's states live in LDS (offsets from rest, one row per
// state) instead of the owners' registers, so that each step can compact the
// slots it solves into a list that all threads share.  Per split step:
//   1. each thread decides for its slots whether they are solved (the last
//      check found the slot or a neighbour in its fiber active, or a
//      stimulus covers one of them; fibers take part from their first
//      stimulus on) with bit masks over a window of the bin's bit-packed
//      verdicts, applies V_m prescriptions and flags the fibers that have a
//      solved slot;
//   2. one LDS atomic per wave reserves list positions for the solved slots
//      (their order in the list does not matter: every slot is solved on
//      its own) -- except slots with a stimulus current, which their owners
//      solve themselves (a handful per fiber), so that the list carries no
//      current;
//   3. the first reaction part runs over the list, T slots at a time, and on
//      the owners' current-stimulated slots (Godunov: the only part, with
//      the equilibrium check);
//   4. the owners run the diffusion on their slots, with a zero right-hand
//      side on fibers without a solved slot (which keeps them exact);
//   5. Strang: the second reaction half and the check, as in 3;
//   6. the owners take the observables of their slots.
// A bin with no slot to solve in a step skips 3-5: its diffusion would have
// a zero right-hand side everywhere.  The point flags come from and go back
// to device memory (one byte per node: PT_ACTIVE), as in the split schedule.
template <int K, int MAXT>
__global__ __launch_bounds__(MAXT) void k_run_hh_adapt(KArgs A) {
  extern __shared__ float lds[];
  const int T = blockDim.x;
  const int t = threadIdx.x;
  const int cap = A.cap;
  const int64_t bslot = (int64_t)blockIdx.x * cap;  // the bin's first slot
  const int s0 = t * K;                              // this thread's first slot in the bin
  const int64_t nt = A.n_total;
  float* s_y = lds + (size_t)T * (6 + 2 * A.pcr_levels);
  uint16_t* s_list = reinterpret_cast<uint16_t*>(s_y + 4 * (size_t)cap);
  uint8_t* s_fib = reinterpret_cast<uint8_t*>(s_list + cap);    // bin-local fiber per slot
  uint32_t* s_act = reinterpret_cast<uint32_t*>(s_fib + cap);   // verdict bits, cap / 32 + 2 words
  const int n_words = cap / 32 + 2;
  uint8_t* s_fany = reinterpret_cast<uint8_t*>(s_act + n_words);  // [2][kBinFibers]
  int32_t* s_cnt = reinterpret_cast<int32_t*>(s_fany + 2 * kBinFibers);  // [2] list lengths
  int32_t* s_any = s_cnt + 2;                                            // [2] anything solved
  const int lane = t & 63;
  const int32_t* first_on = A.bin_first_on + (int64_t)blockIdx.x * kBinFibers;
  constexpr uint32_t allK = (K >= 32) ? 0xffffffffu : ((1u << K) - 1u);

  for (int j = t; j < n_words; j += T) s_act[j] = 0u;
  for (int j = t; j < kBinFibers; j += T) {
    s_fany[j] = 0;
    s_fany[kBinFibers + j] = 0;
  }
  if (t < 2) {
    s_cnt[t] = 0;
    s_any[t] = 0;
  }
  uint32_t info[K];
  float vcur[K];        // V of each slot at the end of the previous step
  uint32_t done = 0;    // slots that need no activation-time update
  uint32_t act0 = 0;    // verdicts of the previous step (for the setup only)
  uint32_t lmask = 0, rmask = 0, smask = 0;  // left / right neighbour in the fiber; stimulus entry
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int sl = s0 + q;
    info[q] = A.slot_info[bslot + sl];
    const int32_t g = A.slot_gidx[bslot + sl];
    if (info[q] & SLOT_L) lmask |= 1u << q;
    if (info[q] & SLOT_R) rmask |= 1u << q;
    if (info[q] >> SLOT_STIM_SHIFT) smask |= 1u << q;
    if (g >= 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) s_y[k * cap + sl] = A.state[k * nt + g];
      s_fib[sl] = A.slot_fiber[bslot + sl];
      if (A.pt_prev[g] & PT_ACTIVE) act0 |= 1u << q;
      if (!isinf(A.t_act[g])) done |= 1u << q;
      vcur[q] = A.state[g];
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) s_y[k * cap + sl] = 0.0f;
      s_fib[sl] = 0;
      done |= 1u << q;
      vcur[q] = 0.0f;
    }
  }
  // slots of fibers that take part, and the next step at which one more of
  // this thread's fibers joins (rare: recomputed then)
  uint32_t onmask = 0;
  int32_t next_on = INT32_MAX;
  auto update_on = [&](int32_t n) {
    onmask = 0;
    next_on = INT32_MAX;
    for (int q = 0; q < K; ++q) {
      if (!(info[q] & SLOT_REAL)) continue;
      const int32_t f1 = first_on[A.slot_fiber[bslot + s0 + q]];
      if (n >= f1) onmask |= 1u << q;
      else next_on = f1 < next_on ? f1 : next_on;
    }
  };
  update_on(A.step0);
  // stimulus entries of the slots next to this thread's first and last
  const uint32_t sid_l = t > 0 ? (A.slot_info[bslot + s0 - 1] >> SLOT_STIM_SHIFT) : 0u;
  const uint32_t sid_r = t + 1 < T ? (A.slot_info[bslot + s0 + K] >> SLOT_STIM_SHIFT) : 0u;
  CNConst<K> cc;
  cn_setup<K>(cc, pack_lr<K>(info), A.r_mat, lds, T, t, A.pcr_levels);  // its barriers order the clears above
  for (uint32_t m = act0; m; m &= m - 1u) {
    const int sl = s0 + __builtin_ctz(m);
    atomicOr(&s_act[sl >> 5], 1u << (sl & 31));
  }
  __syncthreads();
  const hh::Ref ref{A.rest[0], A.rest[1], A.rest[2], A.rest[3]};

  // verdict of slot sl into the bit array
  auto set_verdict = [&](int sl, bool moved) {
    const uint32_t bit = 1u << (sl & 31);
    if (moved)
      atomicOr(&s_act[sl >> 5], bit);
    else
      atomicAnd(&s_act[sl >> 5], ~bit);
  };
  // reaction part of n_s substeps on slot sl with current I; with `check`
  // the equilibrium verdict goes to the bit array
  auto react = [&](int sl, float I, int n_s, bool check) {
    hh::State y{s_y[sl], s_y[cap + sl], s_y[2 * cap + sl], s_y[3 * cap + sl]};
    const hh::State b = y;
    for (int s = 0; s < n_s; ++s) hh::heun(y, I, A.tau, A.inv_cm, ref);
    s_y[sl] = y.V;
    s_y[cap + sl] = y.m;
    s_y[2 * cap + sl] = y.h;
    s_y[3 * cap + sl] = y.n;
    if (check) {
      const float u[4] = {y.V, y.m, y.h, y.n}, ub[4] = {b.V, b.m, b.h, b.n};
      set_verdict(sl, point_moved<4>(u, ub, A.rest, A.adapt_tol));
    }
  };

  const int32_t n_end = A.step0 + A.n_steps;
  unsigned long long solved = 0;
  for (int32_t n = A.step0; n < n_end; ++n) {
    const int par = n & 1;
    if (n >= next_on) update_on(n);
    // 1. slots to solve: a window of verdict bits from slot s0 - 1 to s0 + K
    uint32_t solve, cur = 0;  // cur: solved slots with a stimulus current
    {
      uint64_t win;
      if (t > 0) {
        const int w = (s0 - 1) >> 5;
        win = ((uint64_t)s_act[w] | ((uint64_t)s_act[w + 1] << 32)) >> ((s0 - 1) & 31);
      } else {
        win = ((uint64_t)s_act[0] | ((uint64_t)s_act[1] << 32)) << 1;
      }
      uint32_t hot = (uint32_t)(win >> 1) & allK;  // active, or stimulated now
      for (uint32_t m = smask; m; m &= m - 1u) {
        const int q = __builtin_ctz(m);
        if (stim_any_on(A.slot_info[bslot + s0 + q] >> SLOT_STIM_SHIFT, A.stim, n)) hot |= 1u << q;
      }
      const uint32_t hot_l = t > 0 && ((win & 1u) || stim_any_on(sid_l, A.stim, n)) ? 1u : 0u;
      const uint32_t hot_r =
          t + 1 < T && (((win >> (K + 1)) & 1u) || stim_any_on(sid_r, A.stim, n)) ? 1u : 0u;
      const uint32_t hw = hot_l | (hot << 1) | (hot_r << (K + 1));  // bit q + 1: slot q
      solve = onmask & (hot | (hw & lmask) | ((hw >> 2) & rmask));
      // prescriptions and currents of the solved stimulated slots
      for (uint32_t m = solve & smask; m; m &= m - 1u) {
        const int q = __builtin_ctz(m);
        float I, vp;
        if (stim_eval(A.slot_info[bslot + s0 + q] >> SLOT_STIM_SHIFT, A.stim, n, I, vp))
          s_y[s0 + q] = vp;
        if (I != 0.0f) cur |= 1u << q;
      }
      // one flag per fiber run of solved slots (a fiber starts at a slot
      // without a left neighbour)
      const uint32_t starts = ~lmask & allK;
      for (uint32_t m = solve; m;) {
        const int q = __builtin_ctz(m);
        s_fany[par * kBinFibers + s_fib[s0 + q]] = 1;
        const uint32_t later = starts & ~((2u << q) - 1u);  // fiber starts after q
        m &= later ? ~((1u << __builtin_ctz(later)) - 1u) : 0u;
      }
    }
    // 2. list positions: a wave-level prefix of the counts from one ballot
    // per bit of the count, and one LDS atomic per wave
    const uint32_t listed = solve & ~cur;
    const int cnt = __popc(listed);
    solved += (unsigned)__popc(solve);
    const uint64_t below = (1ull << lane) - 1ull;
    int excl = 0, wave_total = 0;
#pragma unroll
    for (int b = 0; (1 << b) <= K; ++b) {
      const uint64_t bits = __ballot((cnt >> b) & 1);
      excl += __popcll(bits & below) << b;
      wave_total += __popcll(bits) << b;
    }
    int base = 0;
    if (lane == 0 && wave_total > 0) base = atomicAdd(&s_cnt[par], wave_total);
    base = __builtin_amdgcn_readfirstlane(base);
    int pos = base + excl;
    for (uint32_t m = listed; m; m &= m - 1u) s_list[pos++] = (uint16_t)(s0 + __builtin_ctz(m));
    if (solve) s_any[par] = 1;
    // the other parity's counters and fiber flags were last read in the
    // previous step; clear them for the next one
    if (t == 0) {
      s_cnt[par ^ 1] = 0;
      s_any[par ^ 1] = 0;
    }
    for (int j = t; j < kBinFibers; j += T) s_fany[(par ^ 1) * kBinFibers + j] = 0;
    __syncthreads();
    const int total = s_cnt[par];

    if (s_any[par]) {
      uint32_t live = 0;  // slots of fibers with a solved slot
#pragma unroll
      for (int q = 0; q < K; ++q)
        if (s_fany[par * kBinFibers + s_fib[s0 + q]]) live |= 1u << q;
      // 3. first reaction part (Godunov: the only one, checked)
      const bool check_first = A.n_sub2 == 0;
      for (int j = t; j < total; j += T) react(s_list[j], 0.0f, A.n_sub, check_first);
      for (uint32_t m = cur; m; m &= m - 1u) {
        const int sl = s0 + __builtin_ctz(m);
        react(sl, stim_current(A.slot_info[bslot + sl] >> SLOT_STIM_SHIFT, A.stim, n), A.n_sub,
              check_first);
      }
      __syncthreads();
      // 4. diffusion on the fibers with a solved slot
      {
        float V[K];
#pragma unroll
        for (int q = 0; q < K; ++q) V[q] = s_y[s0 + q];
        for (int c = 0; c < A.n_cn; ++c)
          cn_solve<K>(V, pack_lr<K>(info), A.r_mat, A.rhs, cc, lds, T, t, A.pcr_levels, live);
#pragma unroll
        for (int q = 0; q < K; ++q) s_y[s0 + q] = V[q];
      }
      __syncthreads();
      // 5. Strang: second reaction half and the equilibrium check
      if (!check_first) {
        for (int j = t; j < total; j += T) react(s_list[j], 0.0f, A.n_sub2, true);
        for (uint32_t m = cur; m; m &= m - 1u) {
          const int sl = s0 + __builtin_ctz(m);
          react(sl, stim_current(A.slot_info[bslot + sl] >> SLOT_STIM_SHIFT, A.stim, n), A.n_sub2,
                true);
        }
        __syncthreads();
      }
    }

    // 6. observables of this thread's slots
    {
      const float t0 = (float)n * A.dt;
      const float uth = A.v_th - A.rest[0];
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const float v1 = s_y[s0 + q];
        if (!((done >> q) & 1u) && vcur[q] < uth && v1 >= uth) {
          const int32_t g = A.slot_gidx[bslot + s0 + q];
          A.t_act[g] = fmaf(A.dt, (uth - vcur[q]) / (v1 - vcur[q]), t0);
          done |= 1u << q;
        }
        vcur[q] = v1;
      }
    }
    if (A.sample_every > 0 && ((int64_t)n + 1) % A.sample_every == 0) {
      const int64_t row = ((int64_t)n + 1) / A.sample_every - 1 - A.sample_row0;
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const int32_t g = A.slot_gidx[bslot + s0 + q];
        if (g >= 0) A.samples[row * nt + g] = vcur[q] + A.rest[0];
      }
    }
  }

  bool bad = false;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int sl = s0 + q;
    const int32_t g = A.slot_gidx[bslot + sl];
    if (g >= 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float v = s_y[k * cap + sl];
        A.state[k * nt + g] = v;
        bad |= !isfinite(v);
      }
      A.pt_cur[g] = ((s_act[sl >> 5] >> (sl & 31)) & 1u) ? PT_ACTIVE : 0;
    }
  }
  if (bad) atomicOr(A.flag, 1);
  if (solved) atomicAdd(&A.adapt_count[blockIdx.x % kAdaptCounters], solved);
}

// ---------------------------------------------------------------------------
// Diffusion only (states in device memory)
// ---------------------------------------------------------------------------

// Bin entry of slot s: the last entry starting at or before s (s below the
// bin's load; n = entries including the end entry).
__device__ __forceinline__ int bin_entry_of(const int32_t* __restrict__ s0, int n, int s) {
  int lo = 0, hi = n - 2;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s0[mid] <= s) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Entries of bin b (starts, first nodes, fibers, max_ents apart) into buf;
// all threads; returns their number.
__device__ __forceinline__ int bin_entries(const KArgs& A, int b, int32_t* buf, int T, int t) {
  const int32_t e0 = A.bin_ent[b];
  const int ne = A.bin_ent[b + 1] - e0;
  for (int j = t; j < ne; j += T) {
    buf[j] = A.ent_s0[e0 + j];
    buf[A.max_ents + j] = A.ent_gofs[e0 + j];
    buf[2 * A.max_ents + j] = A.ent_fiber[e0 + j];
  }
  return ne;
}

// V of slots t + i T of the bin whose entries are in buf (0 past its load),
// and bit i of `live`: the slot's fiber takes part in the step (always, or
// with adaptive computation when a node of the fiber is solved; padding
// slots take part without adaptive computation, where they have no
// couplings and a zero right-hand side).  Consecutive lanes take
// consecutive slots, i.e. consecutive nodes of one fiber: the loads are
// coalesced.
template <int K>
__device__ __forceinline__ void bin_fetch(const KArgs& A, const int32_t* buf, int ne, int T,
                                          int t, float (&v)[K], uint32_t& live) {
  const int32_t load = buf[ne - 1];
  if (ne == 2) {
    // one fiber: slot s is node buf[me] + s; `live` is the fiber's flag for
    // every real slot
    const float* __restrict__ src = A.state + buf[A.max_ents];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int s = t + i * T;
      v[i] = s < load ? src[s] : 0.0f;
    }
    live = ~0u;
    if (A.fiber_any) {
      const int32_t f = buf[2 * A.max_ents];
      if (!A.fiber_any[f]) live = 0u;
      if (t == 0) A.fiber_any_next[f] = 0;
    }
    return;
  }
  live = 0u;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const int s = t + i * T;
    v[i] = 0.0f;
    if (s < load) {
      const int e = bin_entry_of(buf, ne, s);
      const int32_t s0 = buf[e];
      v[i] = A.state[buf[A.max_ents + e] + (s - s0)];
      if (A.fiber_any) {
        const int32_t f = buf[2 * A.max_ents + e];
        if (A.fiber_any[f]) live |= 1u << i;
        // the fiber's first node clears its flag for the step after next
        if (s == s0) A.fiber_any_next[f] = 0;
      } else {
        live |= 1u << i;
      }
    } else if (!A.fiber_any) {
      live |= 1u << i;
    }
  }
}

// Persistent over bins b = blockIdx.x, + gridDim.x, ...: while one bin is
// solved, the V of the next one (and the entries of the one after) are
// already on their way, so the load latency overlaps the solve's barriers.
// Per bin, V is staged through LDS from the coalesced slot order t + i T to
// the thread-contiguous order t K + q the partitioned solve works in, and
// back for the coalesced stores.
template <int K, int MAXT, bool ONE>
__global__ __launch_bounds__(MAXT) void k_diffusion(KArgs A) {
  extern __shared__ float lds[];
  const int T = blockDim.x;
  const int t = threadIdx.x;
  const int cap = A.cap;
  const int G = gridDim.x;
  const int me = A.max_ents;
  float* sV = lds;                                // staged V of every slot
  uint8_t* sInf = (uint8_t*)(lds + cap);          // SLOT_L | SLOT_R | live << 2
  float* cn = (float*)((char*)lds + diffusion_stage_part(cap));  // the solve's arrays
  int32_t* eb0 = (int32_t*)((char*)lds + diffusion_region_bytes(T, A.pcr_levels, cap));
  int32_t* eb1 = eb0 + 3 * me;
  int b = blockIdx.x;
  if (b >= A.n_bins) return;
  int ne = bin_entries(A, b, eb0, T, t);
  int ne_n = b + G < A.n_bins ? bin_entries(A, b + G, eb1, T, t) : 0;
  __syncthreads();
  float vn[K];
  uint32_t live_n;
  bin_fetch<K>(A, eb0, ne, T, t, vn, live_n);
  for (int j = 0; b < A.n_bins; ++j, b += G) {
    int32_t* cur = (j & 1) ? eb1 : eb0;
    int32_t* nxt = (j & 1) ? eb0 : eb1;
    const int32_t load = cur[ne - 1];
    const bool one = ne == 2;  // one fiber in the bin (uniform)
    if (one) {
#pragma unroll
      for (int i = 0; i < K; ++i) sV[t + i * T] = vn[i];
    } else {
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const int s = t + i * T;
        uint32_t inf = ((live_n >> i) & 1u) << 2;
        if (s < load) {
          const int e = bin_entry_of(cur, ne, s);
          const int32_t s0 = cur[e];
          inf |= (s > s0 ? SLOT_L : 0u) | (s + 1 < cur[e + 1] ? SLOT_R : 0u);
        }
        sV[s] = vn[i];
        sInf[s] = (uint8_t)inf;
      }
    }
    __syncthreads();
    float V[K];
    uint32_t lr = 0u;    // coupling bits, two per slot
    uint32_t live = 0u;  // slots whose fiber takes part
    const float vl = t > 0 ? sV[t * K - 1] : 0.0f;
    const float vr = t + 1 < T ? sV[t * K + K] : 0.0f;
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const int s = t * K + q;
      V[q] = sV[s];
      if (one) {
        // padding slots take part exactly when there is no adaptive
        // computation (live_n is all ones then)
        const bool real = s < load;
        lr |= (real ? ((s > 0 ? SLOT_L : 0u) | (s + 1 < load ? SLOT_R : 0u)) : 0u) << (2 * q);
        live |= ((real || !A.fiber_any) ? (live_n & 1u) : 0u) << q;
      } else {
        const uint32_t bq = sInf[s];
        lr |= (bq & 3u) << (2 * q);
        live |= ((bq >> 2) & 1u) << q;
      }
    }
    // the next bin's V and the entries of the one after it
    const int bn = b + G, bnn = b + 2 * G;
    if (bn < A.n_bins) bin_fetch<K>(A, nxt, ne_n, T, t, vn, live_n);
    int ne_nn = 0;
    int32_t e0nn = 0, r_s0 = 0, r_go = 0, r_f = 0;
    if (bnn < A.n_bins) {
      e0nn = A.bin_ent[bnn];
      ne_nn = A.bin_ent[bnn + 1] - e0nn;
      if (t < ne_nn) {
        r_s0 = A.ent_s0[e0nn + t];
        r_go = A.ent_gofs[e0nn + t];
        r_f = A.ent_fiber[e0nn + t];
      }
    }
    if constexpr (ONE) {  // launched for exactly one substep
      cn_merged<K>(V, vl, vr, lr, A.r_mat, A.rhs, live, cn, cn + 3 * T, cn + 11 * T, T, t,
                   A.pcr_levels);
    } else {
      CNConst<K> cc;
      cn_setup<K>(cc, lr, A.r_mat, cn, T, t, A.pcr_levels);
      for (int c = 0; c < A.n_cn; ++c)
        cn_solve<K>(V, lr, A.r_mat, A.rhs, cc, cn, T, t, A.pcr_levels, live);
    }
    // every read of the staged V (own slots, neighbours) came before the
    // solve's first barrier
#pragma unroll
    for (int q = 0; q < K; ++q) sV[t * K + q] = V[q];
    __syncthreads();
    if (one) {
      float* __restrict__ dst = A.state + cur[me];
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const int s = t + i * T;
        if (s < load) dst[s] = sV[s];
      }
    } else {
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const int s = t + i * T;
        if (s < load) {
          const int e = bin_entry_of(cur, ne, s);
          A.state[cur[me + e] + (s - cur[e])] = sV[s];
        }
      }
    }
    __syncthreads();  // cur and the staging are free
    if (bnn < A.n_bins) {
      if (t < ne_nn) {
        cur[t] = r_s0;
        cur[me + t] = r_go;
        cur[2 * me + t] = r_f;
      }
      for (int jj = t + T; jj < ne_nn; jj += T) {
        cur[jj] = A.ent_s0[e0nn + jj];
        cur[me + jj] = A.ent_gofs[e0nn + jj];
        cur[2 * me + jj] = A.ent_fiber[e0nn + jj];
      }
    }
    ne = ne_n;
    ne_n = ne_nn;
  }
}

// ---------------------------------------------------------------------------
// Reaction with states in device memory, one node per thread
// ---------------------------------------------------------------------------

template <bool APX>
struct ModelHHT {
  static constexpr int S = 4;
  __device__ static void heun(float (&u)[S], const float* ref, float I, float tau, float inv_cm) {
    hh::State y{u[0], u[1], u[2], u[3]};
    const hh::Ref r{ref[0], ref[1], ref[2], ref[3]};
    hh::heun<APX>(y, I, tau, inv_cm, r);
    u[0] = y.V;
    u[1] = y.m;
    u[2] = y.h;
    u[3] = y.n;
  }
};
using ModelHH = ModelHHT<false>;
using ModelHHApx = ModelHHT<true>;

template <bool APX>
struct ModelST57T {
  static constexpr int S = st57::S;
  __device__ static void heun(float (&u)[S], const float* ref, float I, float tau, float inv_cm) {
    st57::heun<APX>(u, ref, I, tau, inv_cm);
  }
};
using ModelST57 = ModelST57T<false>;
// ST57 with exp* and log* (eq. apx-e-function, figure apxlog)
using ModelST57Apx = ModelST57T<true>;

// flags bit 0: reaction with the stimulus of split step `step_a`;
// bit 1: then the observables at the end of split step `step_a`
//        (activation time from v_prev, samples, v_prev := V);
// bit 2: then the start of split step `step_b`: its V_m prescriptions and
//        reaction with its stimulus current.
// The Strang split schedule runs the second half of step n and the first
// half of step n+1 in one launch, so the states cross HBM once per split
// step; the Godunov schedule runs the observables of step n-1 and the
// reaction of step n.
constexpr int REACT_A = 1, REACT_OBSERVE = 2, REACT_B = 4;

// Observables at the end of split step `step` for node i with V_m offset
// v1: activation time from v_prev, the V_m sample of sample steps, then
// v_prev := v1.
// v0 and ta are the node's v_prev and t_act, read by the caller.
__device__ __forceinline__ void observe_step_from(const KArgs& A, int64_t i, int32_t step,
                                                  float v0, float ta, float v1) {
  const float uth = A.v_th - A.rest[0];
  if (isinf(ta) && v0 < uth && v1 >= uth)
    A.t_act[i] = fmaf(A.dt, (uth - v0) / (v1 - v0), (float)step * A.dt);
  if (A.sample_every > 0 && ((int64_t)step + 1) % A.sample_every == 0) {
    const int64_t row = ((int64_t)step + 1) / A.sample_every - 1 - A.sample_row0;
    A.samples[row * A.n_total + i] = v1 + A.rest[0];
  }
  A.v_prev[i] = v1;
  if (!isfinite(v1)) atomicOr(A.flag, 1);
}

__device__ __forceinline__ void observe_step(const KArgs& A, int64_t i, int32_t step, float v1) {
  observe_step_from(A, i, step, A.v_prev[i], A.t_act[i], v1);
}

// The reaction phases of one node (flags as above) on its states u.
template <class M>
__device__ __forceinline__ void react_node(const KArgs& A, int64_t i, float (&u)[M::S],
                                           int32_t step_a, int32_t step_b, int flags) {
  const uint32_t sid = (uint32_t)A.node_stim[i];
  if (flags & REACT_A) {
    const float I = stim_current(sid, A.stim, step_a);
    for (int s = 0; s < A.n_sub; ++s) M::heun(u, A.rest, I, A.tau, A.inv_cm);
  }
  if (flags & REACT_OBSERVE) observe_step(A, i, step_a, u[0]);
  if (flags & REACT_B) {
    float I, vp;
    if (stim_eval(sid, A.stim, step_b, I, vp)) u[0] = vp;
    for (int s = 0; s < A.n_sub; ++s) M::heun(u, A.rest, I, A.tau, A.inv_cm);
  }
}

template <class M>
__global__ __launch_bounds__(256) void k_react(KArgs A, int32_t step_a, int32_t step_b,
                                               int flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n_total) return;
  const int32_t base = step_base_of(A);
  step_a += base;
  step_b += base;
  const int64_t nt = A.n_total;
  float u[M::S];
#pragma unroll
  for (int k = 0; k < M::S; ++k) u[k] = A.state[k * nt + i];
  react_node<M>(A, i, u, step_a, step_b, flags);
#pragma unroll
  for (int k = 0; k < M::S; ++k) A.state[k * nt + i] = u[k];
}

// The same phases over a grid that fits on the device at once: a thread
// takes nodes i, i + stride, ... and loads the next node's states before it
// solves the current one.  A model whose right-hand side holds few waves
// per SIMD (ST57: two, at 242 VGPRs) has little else there to cover the
// loads; this way they run under the wave's own arithmetic.  Loads return in issue order,
// so everything the current node reads (stimulus entry, v_prev, t_act) is
// read before the next node's loads are issued: waiting for it then does
// not wait for them.
template <class M>
__global__ __launch_bounds__(256) void k_react_stream(KArgs A, int32_t step_a, int32_t step_b,
                                                      int flags) {
  const int64_t nt = A.n_total;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const bool obs = flags & REACT_OBSERVE;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  const int32_t base = step_base_of(A);
  step_a += base;
  step_b += base;
  // the next node's inputs: states, stimulus entry, v_prev and t_act
  float nx[M::S];
  uint32_t nsid = (uint32_t)A.node_stim[i];
  float nv0 = obs ? A.v_prev[i] : 0.0f, nta = obs ? A.t_act[i] : 0.0f;
#pragma unroll
  for (int k = 0; k < M::S; ++k) nx[k] = A.state[k * nt + i];
  for (; i < nt; i += stride) {
    float u[M::S];
#pragma unroll
    for (int k = 0; k < M::S; ++k) u[k] = nx[k];
    const uint32_t sid = nsid;
    float v0 = nv0, ta = nta;
    float Ia = 0.0f, Ib = 0.0f, vb = 0.0f;
    int set_b = 0;
    if (flags & REACT_A) Ia = stim_current(sid, A.stim, step_a);
    if (flags & REACT_B) set_b = stim_eval(sid, A.stim, step_b, Ib, vb);
    // all of them in registers here, so no later wait for one of them waits
    // for the next node's loads too
    asm volatile("" : "+v"(Ia), "+v"(Ib), "+v"(vb), "+v"(set_b), "+v"(v0), "+v"(ta));
    const int64_t j = i + stride;
    if (j < nt) {
      nsid = (uint32_t)A.node_stim[j];
      if (obs) {
        nv0 = A.v_prev[j];
        nta = A.t_act[j];
      }
#pragma unroll
      for (int k = 0; k < M::S; ++k) nx[k] = A.state[k * nt + j];
    }
    if (flags & REACT_A)
      for (int s = 0; s < A.n_sub; ++s) M::heun(u, A.rest, Ia, A.tau, A.inv_cm);
    if (obs) observe_step_from(A, i, step_a, v0, ta, u[0]);
    if (flags & REACT_B) {
      if (set_b) u[0] = vb;
      for (int s = 0; s < A.n_sub; ++s) M::heun(u, A.rest, Ib, A.tau, A.inv_cm);
    }
#pragma unroll
    for (int k = 0; k < M::S; ++k) A.state[k * nt + i] = u[k];
  }
}

// ---------------------------------------------------------------------------
// Adaptive computation (split schedule), one node per thread
// ---------------------------------------------------------------------------

// Whether node i is solved in split step `step` (the rules above); nodes of
// fibers left out carry their flags.  With observe_prev, first the
// observables of step - 1.
__device__ __forceinline__ void adapt_decide(const KArgs& A, int64_t i, int32_t step,
                                             int observe_prev, bool& solve, bool& on,
                                             int32_t& f) {
  const int64_t nt = A.n_total;
  if (observe_prev) observe_step(A, i, step - 1, A.state[i]);
  // every flag of the node and its neighbours read at once (no short
  // circuit, whose branches would serialise the loads); a neighbour counts
  // if it exists and lies on the same fiber
  const int64_t il = i > 0 ? i - 1 : i, ir = i + 1 < nt ? i + 1 : i;
  f = A.node_fiber[i];
  const int32_t fl = A.node_fiber[il], fr = A.node_fiber[ir];
  const uint8_t p = A.pt_prev[i], pl = A.pt_prev[il], pr = A.pt_prev[ir];
  const uint32_t sc = (uint32_t)A.node_stim[i], sl = (uint32_t)A.node_stim[il],
                 sr = (uint32_t)A.node_stim[ir];
  on = step >= A.fiber_first_on[f];
  const bool use_l = il != i && fl == f, use_r = ir != i && fr == f;
  const bool act = ((p & PT_ACTIVE) != 0) | (use_l & ((pl & PT_ACTIVE) != 0)) |
                   (use_r & ((pr & PT_ACTIVE) != 0));
  const int stim = (int)stim_any_on(sc, A.stim, step) |
                   ((int)use_l & (int)stim_any_on(sl, A.stim, step)) |
                   ((int)use_r & (int)stim_any_on(sr, A.stim, step));
  solve = on && (act || stim);
  if (!on) A.pt_cur[i] = p;
}

// Start of split step `step`.  A node of a fiber that takes part (step at or
// after the fiber's first stimulus) is solved if the last check found it or
// a neighbour in its fiber active, or a stimulus entry covers it or a
// neighbour; nodes of fibers left out carry their flags.  Every wave adds
// its solved nodes to one of the counters.
template <class M, bool GODUNOV>
__global__ __launch_bounds__(256) void k_adapt_start(KArgs A, int32_t step, int observe_prev) {
  constexpr int S = M::S;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nt = A.n_total;
  const bool real = i < nt;
  bool solve = false, on = false;
  int32_t f = 0;
  if (real) adapt_decide(A, i, step, observe_prev, solve, on, f);
  const uint64_t mask = __ballot(solve);
  if ((threadIdx.x & 63) == 0 && mask)
    atomicAdd(&A.adapt_count[blockIdx.x % kAdaptCounters], (unsigned long long)__popcll(mask));
  if (!real || !on) return;
  if (!solve) {
    A.pt_cur[i] = 0;
    return;
  }
  A.fiber_any[f] = 1;
  float u[S];
#pragma unroll
  for (int k = 0; k < S; ++k) u[k] = A.state[k * nt + i];
  float I, vp;
  if (stim_eval((uint32_t)A.node_stim[i], A.stim, step, I, vp)) u[0] = vp;
  if (GODUNOV) {
    float b[S];
#pragma unroll
    for (int k = 0; k < S; ++k) b[k] = u[k];
    for (int s = 0; s < A.n_sub; ++s) M::heun(u, A.rest, I, A.tau, A.inv_cm);
    A.pt_cur[i] = point_moved<S>(u, b, A.rest, A.adapt_tol) ? PT_ACTIVE : 0;
  } else {
    for (int s = 0; s < A.n_sub; ++s) M::heun(u, A.rest, I, A.tau, A.inv_cm);
    A.pt_cur[i] = PT_SOLVE;
  }
#pragma unroll
  for (int k = 0; k < S; ++k) A.state[k * nt + i] = u[k];
}

// End of Strang split step `step`: second reaction half and equilibrium
// check of the nodes solved in the step, observables of every node.
template <class M>
__global__ __launch_bounds__(256) void k_adapt_finish(KArgs A, int32_t step) {
  constexpr int S = M::S;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nt = A.n_total;
  if (i >= nt) return;
  float v1;
  if (A.pt_cur[i] & PT_SOLVE) {
    float u[S], b[S];
#pragma unroll
    for (int k = 0; k < S; ++k) b[k] = u[k] = A.state[k * nt + i];
    const float I = stim_current((uint32_t)A.node_stim[i], A.stim, step);
    for (int s = 0; s < A.n_sub; ++s) M::heun(u, A.rest, I, A.tau, A.inv_cm);
    A.pt_cur[i] = point_moved<S>(u, b, A.rest, A.adapt_tol) ? PT_ACTIVE : 0;
#pragma unroll
    for (int k = 0; k < S; ++k) A.state[k * nt + i] = u[k];
    v1 = u[0];
  } else {
    v1 = A.state[i];
  }
  observe_step(A, i, step, v1);
}

// The same steps for a model with a heavy right-hand side (ST57), where a
// kernel that both decides and solves holds its register budget even in the
// many waves that solve nothing.  k_adapt_decide takes the decisions of
// k_adapt_start and appends the solved nodes to a list (one atomic per wave);
// k_adapt_solve runs a reaction part over the list only.  The observables
// of a Strang step are taken by the next step's decisions (observe_prev),
// those of a run's last step by k_observe.  Per node the arithmetic is that of
// k_adapt_start / k_adapt_finish.  Each launch of k_adapt_decide also
// clears the other of the two list counters, the one the next step uses.
template <bool GODUNOV>
__global__ __launch_bounds__(256) void k_adapt_decide(KArgs A, int32_t step, int observe_prev,
                                                      int* __restrict__ list,
                                                      int* __restrict__ counts, int slot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool real = i < A.n_total;
  if (blockIdx.x == 0 && threadIdx.x == 0) counts[slot ^ 1] = 0;
  bool solve = false, on = false;
  int32_t f = 0;
  if (real) adapt_decide(A, i, step, observe_prev, solve, on, f);
  const uint64_t mask = __ballot(solve);
  const int lane = threadIdx.x & 63;
  if (mask) {
    const int first = __ffsll((unsigned long long)mask) - 1;
    int base = 0;
    if (lane == first) {
      atomicAdd(&A.adapt_count[blockIdx.x % kAdaptCounters], (unsigned long long)__popcll(mask));
      base = atomicAdd(counts + slot, __popcll(mask));
    }
    base = __shfl(base, first);
    if (solve) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = (int)i;
  }
  if (!real || !on) return;
  if (!solve) {
    A.pt_cur[i] = 0;
    return;
  }
  A.fiber_any[f] = 1;
  if (!GODUNOV) A.pt_cur[i] = PT_SOLVE;
}

// Reaction part of the nodes list[0 .. *count) in split step `step`.
// PHASE 0: start of a Strang step (prescriptions, first half);
// PHASE 1: end of a Strang step (second half, equilibrium check);
// PHASE 2: a Godunov step (prescriptions, reaction, check).
template <class M, int PHASE>
__global__ __launch_bounds__(256) void k_adapt_solve(KArgs A, int32_t step,
                                                     const int* __restrict__ list,
                                                     const int* __restrict__ count) {
  constexpr int S = M::S;
  const int64_t nt = A.n_total;
  const int64_t n = *count;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = list[e];
    float u[S];
#pragma unroll
    for (int k = 0; k < S; ++k) u[k] = A.state[k * nt + i];
    const uint32_t sid = (uint32_t)A.node_stim[i];
    if (PHASE == 1) {
      const float I = stim_current(sid, A.stim, step);
      for (int s = 0; s < A.n_sub; ++s) M::heun(u, A.rest, I, A.tau, A.inv_cm);
      A.pt_cur[i] = state_moved<S>(u, A.state + i, nt, A.rest, A.adapt_tol) ? PT_ACTIVE : 0;
    } else {
      float I, vp;
      if (stim_eval(sid, A.stim, step, I, vp)) u[0] = vp;
      if (PHASE == 2) {
        float b[S];
#pragma unroll
        for (int k = 0; k < S; ++k) b[k] = u[k];
        for (int s = 0; s < A.n_sub; ++s) M::heun(u, A.rest, I, A.tau, A.inv_cm);
        A.pt_cur[i] = point_moved<S>(u, b, A.rest, A.adapt_tol) ? PT_ACTIVE : 0;
      } else {
        for (int s = 0; s < A.n_sub; ++s) M::heun(u, A.rest, I, A.tau, A.inv_cm);
      }
    }
#pragma unroll
    for (int k = 0; k < S; ++k) A.state[k * nt + i] = u[k];
  }
}

// Observables at the end of split step `step` for every node.
__global__ __launch_bounds__(256) void k_observe(KArgs A, int32_t step) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n_total) return;
  observe_step(A, i, step, A.state[i]);
}

// ---------------------------------------------------------------------------
// Initial state and small utilities
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_init(KArgs A, int S, const float* __restrict__ vm_noise,
                                             const float* __restrict__ rel_noise) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n_total) return;
  const int64_t nt = A.n_total;
  for (int k = 0; k < S; ++k) {
    // rest_k (1 + rel) (+ noise for V_m), stored as the offset from rest_k
    float v = rel_noise ? A.rest[k] * rel_noise[k * nt + i] : 0.0f;
    if (k == 0 && vm_noise) v += vm_noise[i];
    A.state[k * nt + i] = v;
  }
  A.t_act[i] = __builtin_inff();
  A.v_prev[i] = A.state[i];
}

// Node-major copies of the state for training data: U[i][k] = state[k][i].
__global__ __launch_bounds__(256) void k_state_rows(const float* __restrict__ state, int64_t nt,
                                                    int S, float* __restrict__ U) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nt * S) return;
  const int64_t i = e / S;
  const int k = (int)(e % S);
  U[e] = state[k * nt + i];
}

// state[k][i] = U[r0 + i][k] for i < n, 0 for n <= i < nt.
__global__ __launch_bounds__(256) void k_rows_to_state(const float* __restrict__ U, int64_t r0,
                                                       int64_t n, int S, float* __restrict__ state,
                                                       int64_t nt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nt * S) return;
  const int64_t i = e / S;
  const int k = (int)(e % S);
  state[k * nt + i] = i < n ? U[(r0 + i) * S + k] : 0.0f;
}

// dU[r0 + i][k] = state[k][i] - U[r0 + i][k] for i < n.
__global__ __launch_bounds__(256) void k_state_minus_rows(const float* __restrict__ state,
                                                          const float* __restrict__ U, int64_t r0,
                                                          int64_t n, int S, int64_t nt,
                                                          float* __restrict__ dU) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * S) return;
  const int64_t i = e / S;
  const int k = (int)(e % S);
  dU[(r0 + i) * S + k] = state[k * nt + i] - U[(r0 + i) * S + k];
}

__global__ __launch_bounds__(64) void k_step_base(int32_t* p, int32_t v, int set) {
  if (threadIdx.x == 0) *p = set ? v : *p + v;
}

__global__ __launch_bounds__(256) void k_fill(float* p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_check_finite(const float* p, int64_t n, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(p[i])) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Instantiations: nodes per thread K with the largest workgroup MAXT the
// launch may use.  A smaller MAXT gives the compiler more registers per
// thread (1024 threads: 128 VGPRs; 768: 168; 512: 256), which the larger K
// need; plan_fits() in the host runtime accepts exactly these pairs.
#define FIB_FOR_EACH_PLAN(X) \
  X(2, 1024) X(3, 1024) X(4, 1024) X(5, 1024) X(6, 1024) X(7, 1024) X(8, 1024) \
  X(7, 768) X(8, 768) X(9, 768) X(10, 768) \
  X(10, 512) X(11, 512) X(12, 512) X(13, 512) X(14, 512)

int plan_max_threads(int K) {
  if (K >= 2 && K <= 8) return 1024;
  if (K >= 9 && K <= 10) return 768;
  if (K >= 11 && K <= 14) return 512;
  return 0;
}

// Picks the instantiation with the smallest MAXT that still holds `threads`.
template <template <int, int> class L>
static hipError_t dispatch_plan(int K, int threads, int groups, size_t lds, const KArgs& a,
                                hipStream_t s) {
  int best = 0;
#define FIB_PICK(KK, MT) \
  if (K == KK && threads <= MT && (best == 0 || MT < best)) best = MT;
  FIB_FOR_EACH_PLAN(FIB_PICK)
#undef FIB_PICK
#define FIB_LAUNCH(KK, MT) \
  if (K == KK && best == MT) return L<KK, MT>::go(groups, threads, lds, a, s);
  FIB_FOR_EACH_PLAN(FIB_LAUNCH)
#undef FIB_LAUNCH
  return hipErrorInvalidValue;
}

template <int K, int MAXT>
struct FusedLaunch {
  static hipError_t go(int groups, int threads, size_t lds, const KArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_run_hh<K, MAXT, false>), dim3(groups), dim3(threads), lds, s, a);
    return hipGetLastError();
  }
};

template <int K, int MAXT>
struct FusedApxLaunch {
  static hipError_t go(int groups, int threads, size_t lds, const KArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_run_hh<K, MAXT, true>), dim3(groups), dim3(threads), lds, s, a);
    return hipGetLastError();
  }
};

template <int K, int MAXT>
struct FusedAdaptLaunch {
  static hipError_t go(int groups, int threads, size_t lds, const KArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_run_hh_adapt<K, MAXT>), dim3(groups), dim3(threads), lds, s, a);
    return hipGetLastError();
  }
};

// Workgroups of a kernel resident on the current device at once for a
// block size and dynamic LDS (queried once per device and shape; 0 if the
// runtime gives no answer).
template <class Kern>
static int resident_blocks(Kern kern, int threads, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, int, size_t>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_tuple(dev, reinterpret_cast<const void*>(kern), threads, lds);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds) != hipSuccess ||
      cus <= 0 || per_cu <= 0)
    return 0;
  return cache[key] = cus * per_cu;
}

template <int K, int MAXT>
struct DiffusionLaunch {
  static hipError_t go(int groups, int threads, size_t lds, const KArgs& a, hipStream_t s) {
    if (a.n_cn == 1) {
      const int res = resident_blocks(k_diffusion<K, MAXT, true>, threads, lds);
      const int grid = res > 0 ? std::min(groups, res) : groups;
      hipLaunchKernelGGL((k_diffusion<K, MAXT, true>), dim3(grid), dim3(threads), lds, s, a);
    } else {
      const int res = resident_blocks(k_diffusion<K, MAXT, false>, threads, lds);
      const int grid = res > 0 ? std::min(groups, res) : groups;
      hipLaunchKernelGGL((k_diffusion<K, MAXT, false>), dim3(grid), dim3(threads), lds, s, a);
    }
    return hipGetLastError();
  }
};

hipError_t launch_run_fused(int model, int K, int groups, int threads, size_t lds,
                            const KArgs& a, hipStream_t s) {
  if (model == 0) return dispatch_plan<FusedLaunch>(K, threads, groups, lds, a, s);
  if (model == 2) return dispatch_plan<FusedApxLaunch>(K, threads, groups, lds, a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_run_fused_adaptive(int K, int groups, int threads, size_t lds,
                                     const KArgs& a, hipStream_t s) {
  return dispatch_plan<FusedAdaptLaunch>(K, threads, groups, lds, a, s);
}

hipError_t launch_diffusion(int K, int groups, int threads, size_t lds, const KArgs& a,
                            hipStream_t s) {
  if (!a.bin_ent || a.cap != threads * K || a.n_bins != groups) return hipErrorInvalidValue;
  lds = std::max(lds, diffusion_lds_bytes(threads, a.pcr_levels, a.cap, a.max_ents));
  return dispatch_plan<DiffusionLaunch>(K, threads, groups, lds, a, s);
}

// Workgroups of k_react_stream<M> resident on the current device at once
// (queried once per device and model; without an answer, one thread per
// node).
template <class M>
static unsigned st57_stream_blocks() {
  static std::mutex mu;
  static unsigned cache[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return ~0u;
  std::lock_guard<std::mutex> lock(mu);
  if (cache[dev] == 0) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_react_stream<M>, 256,
                                                      0) != hipSuccess ||
        cus <= 0 || per_cu <= 0)
      return ~0u;
    cache[dev] = (unsigned)cus * (unsigned)per_cu;
  }
  return cache[dev];
}

hipError_t launch_react(int model, int32_t step_a, int32_t step_b, int flags, const KArgs& a,
                        hipStream_t s) {
  if (a.n_total == 0) return hipSuccess;
  const dim3 grid(blocks_for(a.n_total, 256)), block(256);
  if (model == 0)
    hipLaunchKernelGGL(k_react<ModelHH>, grid, block, 0, s, a, step_a, step_b, flags);
  else if (model == 2)
    hipLaunchKernelGGL(k_react<ModelHHApx>, grid, block, 0, s, a, step_a, step_b, flags);
  else if (model == 1)
    hipLaunchKernelGGL(k_react_stream<ModelST57>,
                       dim3(std::min(grid.x, st57_stream_blocks<ModelST57>())), block, 0, s, a,
                       step_a, step_b, flags);
  else if (model == 3)
    hipLaunchKernelGGL(k_react_stream<ModelST57Apx>,
                       dim3(std::min(grid.x, st57_stream_blocks<ModelST57Apx>())), block, 0, s, a,
                       step_a, step_b, flags);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_adapt_decide(bool godunov, int32_t step, bool observe_prev, int* list,
                              int* counts, int slot, const KArgs& a, hipStream_t s) {
  if (a.n_total == 0) return hipSuccess;
  const dim3 grid(blocks_for(a.n_total, 256)), block(256);
  if (godunov)
    hipLaunchKernelGGL(k_adapt_decide<true>, grid, block, 0, s, a, step, observe_prev ? 1 : 0,
                       list, counts, slot);
  else
    hipLaunchKernelGGL(k_adapt_decide<false>, grid, block, 0, s, a, step, observe_prev ? 1 : 0,
                       list, counts, slot);
  return hipGetLastError();
}

template <int PHASE>
static void adapt_solve_st57(dim3 grid, int32_t step, const int* list, const int* count,
                             const KArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_adapt_solve<ModelST57, PHASE>), grid, dim3(256), 0, s, a, step, list,
                     count);
}

hipError_t launch_adapt_solve(int model, int phase, int32_t step, const int* list,
                              const int* count, const KArgs& a, hipStream_t s) {
  if (a.n_total == 0) return hipSuccess;
  if (model != 1 || phase < 0 || phase > 2) return hipErrorInvalidValue;
  // grid-stride over the list, whose length only the device knows
  const dim3 grid(std::min(blocks_for(a.n_total, 256), 1024u));
  if (phase == 0) adapt_solve_st57<0>(grid, step, list, count, a, s);
  if (phase == 1) adapt_solve_st57<1>(grid, step, list, count, a, s);
  if (phase == 2) adapt_solve_st57<2>(grid, step, list, count, a, s);
  return hipGetLastError();
}

hipError_t launch_observe(int32_t step, const KArgs& a, hipStream_t s) {
  if (a.n_total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_observe, dim3(blocks_for(a.n_total, 256)), dim3(256), 0, s, a, step);
  return hipGetLastError();
}

template <class M>
static hipError_t adapt_start_for(bool godunov, int32_t step, bool observe_prev, const KArgs& a,
                                  hipStream_t s) {
  const dim3 grid(blocks_for(a.n_total, 256)), block(256);
  if (godunov)
    hipLaunchKernelGGL((k_adapt_start<M, true>), grid, block, 0, s, a, step, observe_prev ? 1 : 0);
  else
    hipLaunchKernelGGL((k_adapt_start<M, false>), grid, block, 0, s, a, step, observe_prev ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_adapt_start(int model, bool godunov, int32_t step, bool observe_prev,
                              const KArgs& a, hipStream_t s) {
  if (a.n_total == 0) return hipSuccess;
  if (model == 0) return adapt_start_for<ModelHH>(godunov, step, observe_prev, a, s);
  if (model == 2) return adapt_start_for<ModelHHApx>(godunov, step, observe_prev, a, s);
  return hipErrorInvalidValue;  // ST57: launch_adapt_decide + launch_adapt_solve
}

hipError_t launch_adapt_finish(int model, int32_t step, const KArgs& a, hipStream_t s) {
  if (a.n_total == 0) return hipSuccess;
  const dim3 grid(blocks_for(a.n_total, 256)), block(256);
  if (model == 0)
    hipLaunchKernelGGL(k_adapt_finish<ModelHH>, grid, block, 0, s, a, step);
  else if (model == 2)
    hipLaunchKernelGGL(k_adapt_finish<ModelHHApx>, grid, block, 0, s, a, step);
  else
    return hipErrorInvalidValue;  // ST57: launch_adapt_solve + launch_observe
  return hipGetLastError();
}

hipError_t launch_init(int model, const float* vm_noise, const float* rel_noise, const KArgs& a,
                       hipStream_t s) {
  const int S = (model == 0 || model == 2) ? ModelHH::S
                : (model == 1 || model == 3) ? ModelST57::S : 0;
  if (S == 0) return hipErrorInvalidValue;
  if (a.n_total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_init, dim3(blocks_for(a.n_total, 256)), dim3(256), 0, s, a, S, vm_noise,
                     rel_noise);
  return hipGetLastError();
}

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_state_rows(const float* state, int64_t nt, int S, float* U, hipStream_t s) {
  if (nt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_state_rows, dim3(blocks_for(nt * S, 256)), dim3(256), 0, s, state, nt, S, U);
  return hipGetLastError();
}

hipError_t launch_rows_to_state(const float* U, int64_t r0, int64_t n, int S, float* state,
                                int64_t nt, hipStream_t s) {
  if (nt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rows_to_state, dim3(blocks_for(nt * S, 256)), dim3(256), 0, s, U, r0, n, S,
                     state, nt);
  return hipGetLastError();
}

hipError_t launch_state_minus_rows(const float* state, const float* U, int64_t r0, int64_t n, int S,
                                   int64_t nt, float* dU, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_state_minus_rows, dim3(blocks_for(n * S, 256)), dim3(256), 0, s, state, U,
                     r0, n, S, nt, dU);
  return hipGetLastError();
}

hipError_t launch_step_base(int32_t* p, int32_t v, bool set, hipStream_t s) {
  hipLaunchKernelGGL(k_step_base, dim3(1), dim3(64), 0, s, p, v, set ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_check_finite(const float* p, int64_t n, int* flag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_finite, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, flag);
  return hipGetLastError();
}

}  // namespace fib
