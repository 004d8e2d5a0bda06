// Surrogate split-step kernels (gfx950).
//
// In surrogate mode the split schedule replaces the pair of reaction halves
// that meet between two diffusion steps, R(dt/2) of step n followed by
// R(dt/2) of step n+1, by one implicit-midpoint step of width dt,
//   du* = dt G(y + du*/2, I),
// solved by fixed-point iteration from the network's prediction du:
//   du1 = dt G(y + du/2, I),   du2 = dt G(y + du1/2, I), ...
// The iteration contracts by q = dt |dG/dy| / 2 (about 0.02 for
// Hodgkin-Huxley at dt = 5e-3 ms, up to 0.26 for ST57 at dt = 5e-4 ms), so
// |du1 - du| measures the network's error and the c-th iterate lies within
// about q^c |du1 - du| / (1 - q) of du*.  Hodgkin-Huxley takes two
// iterations (its right-hand side is cheap), ST57 one (its right-hand side
// is most of the step's arithmetic).  A node keeps the last iterate only if
// |du1 - du|_k <= tol * atol_k for every state k; every other node -- and
// every node whose stimulus current changes between the two halves or whose
// V_m is prescribed at the start of step n+1 -- is appended
// to a compacted list that the fallback kernel advances with the plain
// Heun substeps.  The state at the end of step n, which the pair never
// forms, is taken as the midpoint y + du_c/2 of the last iterate du_c for
// the activation-time observable; steps that write V_m samples run the
// plain path everywhere.
//
// Network on the matrix cores, one wave per tile of 64 nodes (lane = node
// for everything outside the network): nodes are the N dimension of
// v_mfma_f32_16x16x32_bf16 (16 nodes per instruction, four node groups per
// tile) and the weights are the A operand, pre-packed in BF16 fragments
// that the workgroup stages in LDS once; every fragment read from LDS
// serves the four groups.  A layer's output D holds, in lane l, features
// 16 ob + 4 (l / 16) + j of node l % 16 of the group; the next layer takes
// its K-block kb from the output blocks 2 kb and 2 kb + 1 of the same lane,
// so activations stay in registers and the weight packing absorbs the
// implied permutation of the K index:
//   K index 8 g + i  <->  feature 32 kb + 4 g + i          (i < 4)
//                          feature 32 kb + 16 + 4 g + i - 4 (i >= 4).
// The node-major network inputs (BF16) and outputs (FP16) pass through a
// per-wave LDS region whose row strides (KIN_PAD + 8 and OUT_PAD + 4
// elements) spread 16-byte row accesses of consecutive lanes over all
// banks; the outputs overwrite the inputs, which are all in registers by
// then.  Biases initialise the accumulators.
#include <mutex>

#include "../../include/fib.h"
#include "fib_internal.h"
#include "hh_model.h"
#include "st57_model.h"
#include "surrogate_internal.h"

namespace fib {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Feature of the previous layer feeding K index (kb, lane group g, element i).
__host__ __device__ inline int k_feature(bool first, int kb, int g, int i) {
  if (first) return 32 * kb + 8 * g + i;
  return i < 4 ? 32 * kb + 4 * g + i : 32 * kb + 16 + 4 * g + (i - 4);
}

// Packs FP32 master parameters (flat layout) into the BF16 fragments and
// FP32 biases of a SurrogateNet.  One thread per fragment element.
__global__ __launch_bounds__(256) void k_pack(SurrogateNet net, const float* __restrict__ params,
                                              __bf16* __restrict__ frags,
                                              float* __restrict__ biases) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < net.frag_elems) {
    // locate layer
    int l = 1;
    while (l < net.L && e >= (int64_t)net.frag_off[l + 1] * 512) ++l;
    const int64_t le = e - (int64_t)net.frag_off[l] * 512;
    const int frag = (int)(le / 512), within = (int)(le % 512);
    const int lane = within / 8, i = within % 8;
    const int kblocks = net.pad_in[l] / 32;
    const int ob = frag / kblocks, kb = frag % kblocks;
    const int out = 16 * ob + (lane & 15);
    const int in = k_feature(l == 1, kb, lane >> 4, i);
    float w = 0.0f;
    if (out < net.n_out[l] && in < net.n_in[l]) w = params[net.w_off[l] + out * net.n_in[l] + in];
    frags[e] = (__bf16)w;
  }
  if (e < net.bias_elems) {
    int l = 1;
    while (l < net.L && e >= net.bias_off[l + 1]) ++l;
    const int j = (int)(e - net.bias_off[l]);
    biases[e] = j < net.n_out[l] ? params[net.b_off[l] + j] : 0.0f;
  }
}

typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef short v2s __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef _Float16 v2h __attribute__((ext_vector_type(2)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float silu_fast(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

// Hidden activation of two pre-activations, packed as two BF16 values.
// ReLU acts on the packed BF16 bits: as 16-bit integers, negative BF16
// values (sign bit set) are negative, so max(bits, 0) is ReLU exactly.
template <int ACT>
__device__ __forceinline__ unsigned act_pack(float a, float b) {
  if constexpr (ACT == FIB_ACT_RELU) {
    const v2bf p = __builtin_convertvector((v2f){a, b}, v2bf);
    const v2s m = __builtin_elementwise_max(__builtin_bit_cast(v2s, p), (v2s){0, 0});
    return __builtin_bit_cast(unsigned, m);
  } else {
    const v2bf p = __builtin_convertvector((v2f){silu_fast(a), silu_fast(b)}, v2bf);
    return __builtin_bit_cast(unsigned, p);
  }
}

__device__ __forceinline__ unsigned pack_bf16(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector((v2f){a, b}, v2bf));
}

__device__ __forceinline__ unsigned pack_f16(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector((v2f){a, b}, v2h));
}

// Model adapters: number of states, offsets -> increments of one Heun step.
struct SurHH {
  static constexpr int S = 4;
  __device__ static void rhs_abs(const float (&y)[S], float I, float inv_cm, float (&d)[S]) {
    const hh::State g = hh::rhs(hh::State{y[0], y[1], y[2], y[3]}, I, inv_cm,
                                hh::Ref{0.0f, 0.0f, 0.0f, 0.0f});
    d[0] = g.V;
    d[1] = g.m;
    d[2] = g.h;
    d[3] = g.n;
  }
  __device__ static void rhs(const float (&u)[S], const float* ref, float I, float inv_cm,
                             float (&d)[S]) {
    const hh::State y{u[0], u[1], u[2], u[3]};
    const hh::Ref r{ref[0], ref[1], ref[2], ref[3]};
    const hh::State g = hh::rhs(y, I, inv_cm, r);
    d[0] = g.V;
    d[1] = g.m;
    d[2] = g.h;
    d[3] = g.n;
  }
  __device__ static void heun(float (&u)[S], const float* ref, float I, float tau, float inv_cm) {
    hh::State y{u[0], u[1], u[2], u[3]};
    const hh::Ref r{ref[0], ref[1], ref[2], ref[3]};
    hh::heun(y, I, tau, inv_cm, r);
    u[0] = y.V;
    u[1] = y.m;
    u[2] = y.h;
    u[3] = y.n;
  }
};

struct SurST57 {
  static constexpr int S = st57::S;
  __device__ static void rhs_abs(const float (&y)[S], float I, float inv_cm, float (&d)[S]) {
    st57::rhs_abs<float>(y, I, inv_cm, d);
  }
  __device__ static void rhs(const float (&u)[S], const float* ref, float I, float inv_cm,
                             float (&d)[S]) {
    st57::rhs<float>(u, ref, I, inv_cm, d);
  }
  __device__ static void heun(float (&u)[S], const float* ref, float I, float tau, float inv_cm) {
    st57::heun(u, ref, I, tau, inv_cm);
  }
};

// Walks the S columns of the state array at one node: the column stride
// n_total is added to a pointer held in a vector register and hidden from
// the optimizer, which would otherwise keep all S 64-bit column offsets in
// scalar registers across the persistent loop (hundreds for ST57).  The
// pointer is typed global (address space 1): through a generic pointer the
// accesses compile to flat instructions, which also count against the LDS
// wait counter, so LDS waits would wait for outstanding state loads and
// stores as well (3-4 % of the ST57 step).
struct Column {
  gfloat* p;
  int64_t stride;
  __device__ __forceinline__ Column(const float* q, int64_t s)
      : p((gfloat*)const_cast<float*>(q)), stride(s) {}
  __device__ __forceinline__ void next() {
    p += stride;
    __asm__("" : "+v"(p));
  }
};

// Observables at the end of split step `step` from V offset v1 (the same
// rules as the plain reaction kernel), given the node's V offset v0 at the
// end of the previous step, its activation time t0 so far and the threshold
// offset uth = v_th - rest_V.
__device__ __forceinline__ void observe_with(const KArgs& A, int64_t i, int32_t step, float v1,
                                             float v0, float t0, float uth) {
  if (isinf(t0) && v0 < uth && v1 >= uth)
    A.t_act[i] = fmaf(A.dt, (uth - v0) / (v1 - v0), (float)step * A.dt);
  A.v_prev[i] = v1;
  if (!isfinite(v1)) atomicOr(A.flag, 1);
}

__device__ __forceinline__ void observe(const KArgs& A, int64_t i, int32_t step, float v1) {
  observe_with(A, i, step, v1, A.v_prev[i], A.t_act[i], A.v_th - A.rest[0]);
}

template <int KIN_PAD, int OUT_PAD>
struct Stage {
  static constexpr int XS = KIN_PAD + 8;  // BF16 elements per input row
  static constexpr int OS = OUT_PAD + 4;  // FP16 elements per output row
  static constexpr int kBytes = 64 * XS * 2 > 64 * OS * 2 ? 64 * XS * 2 : 64 * OS * 2;
  static_assert(kBytes % 16 == 0, "stage alignment");
};

// The network for the 64 nodes of one tile: inputs from the wave's stage
// (rows of XS BF16), outputs back to the same stage (rows of OS FP16).
// The four node groups go through in passes of NG groups; each weight
// fragment read from LDS serves the NG groups of a pass (NG = 4 needs the
// most registers, NG = 1 reads every fragment four times).
template <int KIN_PAD, int H, int NHID, int OUT_PAD, int ACT, int NG>
__device__ __forceinline__ void wave_network(char* stage, const v8bf* __restrict__ frag,
                                             const float* __restrict__ wb, const SurrogateNet& net,
                                             int lane) {
  using St = Stage<KIN_PAD, OUT_PAD>;
  constexpr int KB0 = KIN_PAD / 32;  // K-blocks of the input layer
  constexpr int HB = H / 16;         // output blocks of a hidden layer
  constexpr int KBH = H / 32;        // K-blocks of a layer fed by a hidden layer
  constexpr int OB = OUT_PAD / 16;   // output blocks of the last layer
  static_assert(4 % NG == 0, "groups per pass");
  const int r = lane & 15, g = lane >> 4;
  const __bf16* X = reinterpret_cast<const __bf16*>(stage);
  _Float16* O = reinterpret_cast<_Float16*>(stage);

  // all inputs of the tile to registers first: the outputs overwrite them
  v8bf bin[4][KB0];
#pragma unroll
  for (int grp = 0; grp < 4; ++grp)
#pragma unroll
    for (int kb = 0; kb < KB0; ++kb)
      bin[grp][kb] = *reinterpret_cast<const v8bf*>(X + (16 * grp + r) * St::XS + 32 * kb + 8 * g);
  __builtin_amdgcn_wave_barrier();

#pragma unroll
  for (int pass = 0; pass < 4 / NG; ++pass) {
    v4f acc[NG][HB];
#pragma unroll
    for (int ob = 0; ob < HB; ++ob) {
      const v4f bias = *reinterpret_cast<const v4f*>(wb + net.bias_off[1] + 16 * ob + 4 * g);
#pragma unroll
      for (int q = 0; q < NG; ++q) acc[q][ob] = bias;
#pragma unroll
      for (int kb = 0; kb < KB0; ++kb) {
        const v8bf a = frag[(net.frag_off[1] + ob * KB0 + kb) * 64 + lane];
#pragma unroll
        for (int q = 0; q < NG; ++q)
          acc[q][ob] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bin[pass * NG + q][kb], acc[q][ob],
                                                               0, 0, 0);
      }
    }
#pragma unroll
    for (int hl = 0; hl < NHID; ++hl) {
      // activation of hidden layer hl + 1, packed into the next layer's B operands
      v8bf b[NG][KBH];
#pragma unroll
      for (int q = 0; q < NG; ++q)
#pragma unroll
        for (int kb = 0; kb < KBH; ++kb) {
          const v4f lo = acc[q][2 * kb], hi = acc[q][2 * kb + 1];
          const v4u w = {act_pack<ACT>(lo[0], lo[1]), act_pack<ACT>(lo[2], lo[3]),
                         act_pack<ACT>(hi[0], hi[1]), act_pack<ACT>(hi[2], hi[3])};
          b[q][kb] = __builtin_bit_cast(v8bf, w);
        }
      const int layer = hl + 2;
      if (hl + 1 < NHID) {
#pragma unroll
        for (int ob = 0; ob < HB; ++ob) {
          const v4f bias = *reinterpret_cast<const v4f*>(wb + net.bias_off[layer] + 16 * ob + 4 * g);
#pragma unroll
          for (int q = 0; q < NG; ++q) acc[q][ob] = bias;
#pragma unroll
          for (int kb = 0; kb < KBH; ++kb) {
            const v8bf a = frag[(net.frag_off[layer] + ob * KBH + kb) * 64 + lane];
#pragma unroll
            for (int q = 0; q < NG; ++q)
              acc[q][ob] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[q][kb], acc[q][ob], 0, 0, 0);
          }
        }
      } else {
#pragma unroll
        for (int ob = 0; ob < OB; ++ob) {
          const v4f bias = *reinterpret_cast<const v4f*>(wb + net.bias_off[layer] + 16 * ob + 4 * g);
          v4f out[NG];
#pragma unroll
          for (int q = 0; q < NG; ++q) out[q] = bias;
#pragma unroll
          for (int kb = 0; kb < KBH; ++kb) {
            const v8bf a = frag[(net.frag_off[layer] + ob * KBH + kb) * 64 + lane];
#pragma unroll
            for (int q = 0; q < NG; ++q)
              out[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[q][kb], out[q], 0, 0, 0);
          }
#pragma unroll
          for (int q = 0; q < NG; ++q) {
            const uint2 v = {pack_f16(out[q][0], out[q][1]), pack_f16(out[q][2], out[q][3])};
            *reinterpret_cast<uint2*>(O + (16 * (pass * NG + q) + r) * St::OS + 16 * ob + 4 * g) = v;
          }
        }
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// Surrogate reaction pair for every node: finishes step `step_a` and
// starts step `step_a + 1`.  Rejected nodes are appended to list[] through
// count[slot] (one atomic per wave); the kernel clears count[slot ^ 1],
// which the next surrogate step uses, so no separate reset is launched.  With `pred` set, the kernel only writes
// the predicted increments du ([S][n_total]) and changes no state.
// Persistent: each wave walks the 64-node tiles tile = wave_id,
// wave_id + waves, ...  Launch: 64 WAVES threads.
template <class M, int KIN_PAD, int H, int NHID, int OUT_PAD, int ACT, int WAVES, int NG,
          int NCORR>
__global__ __launch_bounds__(64 * WAVES) void k_surrogate(
    KArgs A, SurrogateNet net, const __bf16* __restrict__ frags, const float* __restrict__ biases,
    const float* __restrict__ tab_g, SurrogateScales sc, int32_t step_a, int* __restrict__ list,
    int* __restrict__ counts, int slot, float* __restrict__ pred) {
  extern __shared__ float lds_f[];
  using St = Stage<KIN_PAD, OUT_PAD>;
  constexpr int S = M::S;
  v8bf* wfr = reinterpret_cast<v8bf*>(lds_f);
  float* wb = lds_f + net.frag_elems / 2;
  float* tab = wb + net.bias_elems;
  char* stage_base = reinterpret_cast<char*>(tab + kSurTabFloats);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  char* stage = stage_base + wave * St::kBytes;
  // each lane's (v_prev, t_act), loaded with the tile's states and read back
  // by the observables after the corrector, and the threshold offset: kept
  // in LDS because with ST57 no register is free across the network (in
  // registers they were spilled to scratch, whose reload waits for every
  // outstanding load and store of the wave)
  float2* obs = reinterpret_cast<float2*>(stage_base + WAVES * St::kBytes) + wave * 64;
  float* uth_lds = reinterpret_cast<float*>(stage_base + WAVES * (St::kBytes + 64 * sizeof(float2)));

  {
    const uint4* src = reinterpret_cast<const uint4*>(frags);
    uint4* dst = reinterpret_cast<uint4*>(wfr);
    for (int e = threadIdx.x; e < net.frag_elems / 8; e += 64 * WAVES) dst[e] = src[e];
    for (int e = threadIdx.x; e < net.bias_elems; e += 64 * WAVES) wb[e] = biases[e];
    // the input table (the corrector's tables are read as scalars)
    for (int e = threadIdx.x; e < kTabMid; e += 64 * WAVES) tab[e] = tab_g[e];
    if (threadIdx.x == 0) *uth_lds = A.v_th - A.rest[0];
  }
  __syncthreads();
  int* count = counts ? counts + slot : nullptr;
  if (counts && blockIdx.x == 0 && threadIdx.x == 0) counts[slot ^ 1] = 0;
  const float2* tin = reinterpret_cast<const float2*>(tab + kTabIn);  // scale, bias
  // The corrector's per-state tables are the same for every lane: they are
  // read through the scalar cache (constant address space), not as LDS
  // broadcasts, which moved 20 bytes per state and lane through the LDS
  // next to the weight fragments.  The input table stays in LDS: as scalars
  // its fused multiply-adds would each need a register move.
  typedef __attribute__((address_space(4))) const float cfloat;
  cfloat* tc = (cfloat*)tab_g;
  auto tmid = [&](int k) {  // scale/2, shift/2 + rest
    return make_float2(tc[kTabMid + 2 * k], tc[kTabMid + 2 * k + 1]);
  };
  auto tchk = [&](int k) {  // scale, shift, thr, rest
    return make_float4(tc[kTabChk + 4 * k], tc[kTabChk + 4 * k + 1], tc[kTabChk + 4 * k + 2],
                       tc[kTabChk + 4 * k + 3]);
  };

  const int64_t nt = A.n_total;
  const int64_t tiles = (nt + 63) / 64;
  step_a += step_base_of(A);
  const int32_t step_b = step_a + 1;
  const float span = 2.0f * A.tau * (float)A.n_sub;
  for (int64_t tile = (int64_t)blockIdx.x * WAVES + wave; tile < tiles;
       tile += (int64_t)gridDim.x * WAVES) {
    const int64_t i = tile * 64 + lane;
    const bool real = i < nt;
    // lanes past the end read the last node (their results are dropped)
    const int64_t ic = real ? i : nt - 1;
    // every load of the tile is issued before the first wait: the stimulus
    // id, the observables' inputs and the states (the stimulus evaluation
    // then waits for the id alone)
    const uint32_t sid = (uint32_t)A.node_stim[ic];
    obs[lane] = make_float2(A.v_prev[ic], A.t_act[ic]);
    // this lane's node: offsets in registers for the whole tile
    float u[S];
    {
      Column col{A.state + ic, nt};
#pragma unroll
      for (int k = 0; k < S; ++k) {
        u[k] = *col.p;
        col.next();
      }
    }
    float Ia = 0.0f, Ib = 0.0f;
    bool pres_b = false;  // V_m prescribed at the start of step_b: plain path
    {
      float vp;
      Ia = stim_current(sid, A.stim, step_a);
      pres_b = stim_eval(sid, A.stim, step_b, Ib, vp);
    }
    // network inputs, one 16-byte row chunk at a time
    {
      __bf16* X = reinterpret_cast<__bf16*>(stage);
#pragma unroll
      for (int q = 0; q < KIN_PAD / 8; ++q) {
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = 8 * q + e;
          x[e] = 0.0f;
          if (k < S) {
            const float2 t = tin[k];
            x[e] = fmaf(u[k], t.x, t.y);
          } else if (k == S) {
            x[e] = sc.n_in > S ? Ia * sc.flag_scale : 0.0f;
          }
        }
        const v4u w = {pack_bf16(x[0], x[1]), pack_bf16(x[2], x[3]), pack_bf16(x[4], x[5]),
                       pack_bf16(x[6], x[7])};
        *reinterpret_cast<v4u*>(X + lane * St::XS + 8 * q) = w;
      }
    }
    __builtin_amdgcn_wave_barrier();
    // the matrix-core phase at raised issue priority: with two waves per
    // SIMD, the other wave's vector work then fills the gaps of this one's
    // matrix-core chain instead of delaying it (2-3 % of the ST57 step)
    __builtin_amdgcn_s_setprio(1);
    wave_network<KIN_PAD, H, NHID, OUT_PAD, ACT, NG>(stage, wfr, wb, net, lane);
    __builtin_amdgcn_s_setprio(0);
    // this lane's network outputs, four FP16 values per LDS read
    const v4h* O4 = reinterpret_cast<const v4h*>(reinterpret_cast<const _Float16*>(stage) + lane * St::OS);
    auto out = [&](int k) { return (float)O4[k >> 2][k & 3]; };

    if (pred) {
      if (real) {
        Column col{pred + i, nt};
#pragma unroll
        for (int k = 0; k < S; ++k) {
          const float4 t = tchk(k);
          col.p[0] = fmaf(out(k), t.x, t.y);
          col.next();
        }
      }
      __builtin_amdgcn_wave_barrier();
      continue;
    }

    // fixed-point iterations of the implicit midpoint rule from the
    // prediction; the first one decides acceptance
    bool ok = false;
    if (real) {
      float y[S], G[S];
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const float2 t = tmid(k);
        y[k] = fmaf(out(k), t.x, u[k] + t.y);  // rest + u + du / 2
      }
      M::rhs_abs(y, Ia, A.inv_cm, G);
      // a comparison with NaN is false: a non-finite prediction is rejected
      bool within = true;
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const float4 t = tchk(k);
        const float du = fmaf(out(k), t.x, t.y);
        within &= fabsf(fmaf(span, G[k], -du)) <= t.z;
      }
      const bool flag_ok = sc.n_in > S || Ia == 0.0f;
      ok = within && flag_ok && Ia == Ib && !pres_b;
      if (ok) {
#pragma unroll
        for (int c = 1; c < NCORR; ++c) {
#pragma unroll
          for (int k = 0; k < S; ++k) y[k] = fmaf(0.5f * span, G[k], u[k]) + tchk(k).w;
          M::rhs_abs(y, Ia, A.inv_cm, G);
        }
        const float2 ob = obs[lane];
        observe_with(A, i, step_a, fmaf(0.5f * span, G[0], u[0]), ob.x, ob.y, *uth_lds);
        Column col{A.state + i, nt};
#pragma unroll
        for (int k = 0; k < S; ++k) {
          col.p[0] = fmaf(span, G[k], u[k]);
          col.next();
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    // compaction of the rejected nodes: one atomic per wave
    const bool reject = real && !ok;
    const uint64_t mask = __ballot(reject);
    if (mask) {
      const int first = __ffsll((unsigned long long)mask) - 1;
      int base = 0;
      if (lane == first) base = atomicAdd(count, __popcll(mask));
      base = __shfl(base, first);
      if (reject) {
        const int below = __popcll(mask & ((1ull << lane) - 1ull));
        list[base + below] = (int)i;
      }
    }
  }
}

// The same step with a closed-form predictor instead of the network, as the
// baseline the network is measured against: du = 0 (PRED_ZERO), or the
// explicit Euler increment du = dt G(y, I) (PRED_EULER, one more right-hand
// side), then the corrector iterations, the acceptance test and the
// compaction of the rejected nodes exactly as in k_surrogate.  With the
// zero guess the first iterate is dt G(y) and the test accepts a node only
// if its whole increment is within the tolerance; with the Euler guess the
// first iterate is the explicit midpoint (second-order Runge-Kutta)
// increment and the test bounds its difference to Euler.  The stimulus
// enters G, so stimulated nodes need no flag input.
//
// Streamed like the plain reaction kernel: a grid resident at once, each
// wave takes 64 consecutive nodes per round and issues the loads of its
// next round (states, stimulus entry, v_prev, t_act) before it solves the
// current one.  Every lane of a wave runs the same rounds (lanes past the
// end read the last node and drop their results), so the ballot below sees
// whole waves.  Launch: 256 threads.
template <class M, int PRED, int NCORR>
__global__ __launch_bounds__(256, 2) void k_midpoint(KArgs A, const float* __restrict__ tab_g,
                                                  int32_t step_a, int* __restrict__ list,
                                                  int* __restrict__ counts, int slot) {
  constexpr int S = M::S;
  __shared__ float2 tchk[S];  // (tol res_k, rest_k)
  for (int k = threadIdx.x; k < S; k += 256) {
    const float4 t = reinterpret_cast<const float4*>(tab_g + kTabChk)[k];
    tchk[k] = make_float2(t.z, t.w);
  }
  __syncthreads();
  int* count = counts + slot;
  if (blockIdx.x == 0 && threadIdx.x == 0) counts[slot ^ 1] = 0;
  const int64_t nt = A.n_total;
  step_a += step_base_of(A);
  const int32_t step_b = step_a + 1;
  const float span = 2.0f * A.tau * (float)A.n_sub;
  const float uth = A.v_th - A.rest[0];
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i - lane >= nt) return;  // whole wave past the end
  // the next round's inputs
  float nx[S];
  int64_t ic = i < nt ? i : nt - 1;
  uint32_t nsid = (uint32_t)A.node_stim[ic];
  float nv0 = A.v_prev[ic], nta = A.t_act[ic];
#pragma unroll
  for (int k = 0; k < S; ++k) nx[k] = A.state[k * nt + ic];
  for (; i - lane < nt; i += stride) {
    const bool real = i < nt;
    float u[S];
#pragma unroll
    for (int k = 0; k < S; ++k) u[k] = nx[k];
    const uint32_t sid = nsid;
    float v0 = nv0, ta = nta;
    float Ia = stim_current(sid, A.stim, step_a), Ib, vp;
    int pres_b = stim_eval(sid, A.stim, step_b, Ib, vp);
    // in registers before the next round's loads are issued, so no later
    // wait for one of them waits for those too
    asm volatile("" : "+v"(Ia), "+v"(Ib), "+v"(pres_b), "+v"(v0), "+v"(ta));
    const int64_t j = i + stride;
    if (j - lane < nt) {
      const int64_t jc = j < nt ? j : nt - 1;
      nsid = (uint32_t)A.node_stim[jc];
      nv0 = A.v_prev[jc];
      nta = A.t_act[jc];
#pragma unroll
      for (int k = 0; k < S; ++k) nx[k] = A.state[k * nt + jc];
    }
    float y[S], G[S], du[S];
    if constexpr (PRED == FIB_PRED_EULER) {
#pragma unroll
      for (int k = 0; k < S; ++k) y[k] = u[k] + tchk[k].y;
      M::rhs_abs(y, Ia, A.inv_cm, G);
#pragma unroll
      for (int k = 0; k < S; ++k) du[k] = span * G[k];
    } else {
#pragma unroll
      for (int k = 0; k < S; ++k) du[k] = 0.0f;
    }
#pragma unroll
    for (int k = 0; k < S; ++k) y[k] = fmaf(0.5f, du[k], u[k]) + tchk[k].y;
    M::rhs_abs(y, Ia, A.inv_cm, G);
    bool within = true;
#pragma unroll
    for (int k = 0; k < S; ++k) within &= fabsf(fmaf(span, G[k], -du[k])) <= tchk[k].x;
    const bool ok = real && within && Ia == Ib && !pres_b;
    if (ok) {
#pragma unroll
      for (int c = 1; c < NCORR; ++c) {
#pragma unroll
        for (int k = 0; k < S; ++k) y[k] = fmaf(0.5f * span, G[k], u[k]) + tchk[k].y;
        M::rhs_abs(y, Ia, A.inv_cm, G);
      }
      // observables at the end of step_a from the midpoint
      const float v1 = fmaf(0.5f * span, G[0], u[0]);
      if (isinf(ta) && v0 < uth && v1 >= uth)
        A.t_act[i] = fmaf(A.dt, (uth - v0) / (v1 - v0), (float)step_a * A.dt);
      A.v_prev[i] = v1;
      if (!isfinite(v1)) atomicOr(A.flag, 1);
#pragma unroll
      for (int k = 0; k < S; ++k) A.state[k * nt + i] = fmaf(span, G[k], u[k]);
    }
    const bool reject = real && !ok;
    const uint64_t mask = __ballot(reject);
    if (mask) {
      const int first = __ffsll((unsigned long long)mask) - 1;
      int b = 0;
      if (lane == first) b = atomicAdd(count, __popcll(mask));
      b = __shfl(b, first);
      if (reject) list[b + __popcll(mask & ((1ull << lane) - 1ull))] = (int)i;
    }
  }
}

// Plain reaction pair (second half of step_a, observables, then the start of
// step_a + 1: its V_m prescription and first half) for the nodes in
// list[0..count).  Grid-stride loop, so the grid does not depend on the
// count.  The count is added to *total (nullable), the running number of
// rejections.
template <class M>
__global__ __launch_bounds__(256) void k_fallback(KArgs A, const int* __restrict__ list,
                                                  const int* __restrict__ count, int32_t step_a,
                                                  unsigned long long* __restrict__ total) {
  constexpr int S = M::S;
  const int n = *count;
  if (total && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(total, (unsigned long long)n);
  const int64_t nt = A.n_total;
  step_a += step_base_of(A);
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    const int64_t i = list[e];
    float u[S];
#pragma unroll
    for (int k = 0; k < S; ++k) u[k] = A.state[k * nt + i];
    const uint32_t sid = (uint32_t)A.node_stim[i];
    const float Ia = stim_current(sid, A.stim, step_a);
    for (int s = 0; s < A.n_sub; ++s) M::heun(u, A.rest, Ia, A.tau, A.inv_cm);
    observe(A, i, step_a, u[0]);
    float Ib, vp;
    if (stim_eval(sid, A.stim, step_a + 1, Ib, vp)) u[0] = vp;
    for (int s = 0; s < A.n_sub; ++s) M::heun(u, A.rest, Ib, A.tau, A.inv_cm);
#pragma unroll
    for (int k = 0; k < S; ++k) A.state[k * nt + i] = u[k];
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_pack(const SurrogateNet& net, const float* params, __bf16* frags, float* biases,
                       hipStream_t s) {
  const int64_t n = net.frag_elems > net.bias_elems ? net.frag_elems : net.bias_elems;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, net, params,
                     frags, biases);
  return hipGetLastError();
}

// Kernel configurations: Hodgkin-Huxley 4|5 -> 64 -> 64 -> 64 -> 4 with
// four waves per workgroup (three workgroups fit one CU's LDS), all four
// node groups per weight fragment and two corrector iterations; ST57
// 57|58 -> 128 -> 128 -> 57 with eight waves per workgroup (the 64 KB of
// weights in LDS allow one workgroup per CU, and eight waves keep two per
// SIMD within 256 VGPRs), two node groups per weight fragment and one
// corrector iteration.  Measured on 400 x 1481 ST57 nodes: four waves per
// workgroup (one per SIMD) ran 1.6x slower.
template <class M> struct SurCfg;
template <> struct SurCfg<SurHH> {
  static constexpr int KIN_PAD = 32, H = 64, NHID = 3, OUT_PAD = 16, WAVES = 4, NG = 4, NCORR = 2;
};
#ifndef FIB_SUR_ST57_WAVES
#define FIB_SUR_ST57_WAVES 8
#endif
#ifndef FIB_SUR_ST57_NG
#define FIB_SUR_ST57_NG 2
#endif
#ifndef FIB_SUR_ST57_NCORR
#define FIB_SUR_ST57_NCORR 1
#endif
template <> struct SurCfg<SurST57> {
  static constexpr int KIN_PAD = 64, H = 128, NHID = 2, OUT_PAD = 64;
  static constexpr int WAVES = FIB_SUR_ST57_WAVES, NG = FIB_SUR_ST57_NG,
                       NCORR = FIB_SUR_ST57_NCORR;
};

template <class M>
static size_t sur_lds(const SurrogateNet& net) {
  using C = SurCfg<M>;
  return (size_t)net.frag_elems * 2 + (size_t)net.bias_elems * 4 +
         (size_t)kSurTabFloats * 4 +
         (size_t)C::WAVES * (Stage<C::KIN_PAD, C::OUT_PAD>::kBytes + 64 * sizeof(float2)) +
         sizeof(float);
}

template <class M, int ACT>
static hipError_t sur_launch(const KArgs& a, const SurrogateNet& net, const __bf16* frags,
                             const float* biases, const float* tab, const SurrogateScales& sc,
                             int32_t step_a, int* list, int* counts, int slot, float* pred,
                             unsigned long long* total, hipEvent_t mid, int grid, hipStream_t s) {
  using C = SurCfg<M>;
  const size_t lds = sur_lds<M>(net);
  const int64_t tiles = (a.n_total + 63) / 64;
  const int64_t need = (tiles + C::WAVES - 1) / C::WAVES;
  const unsigned blocks = (unsigned)(need < grid ? need : grid);
  hipLaunchKernelGGL((k_surrogate<M, C::KIN_PAD, C::H, C::NHID, C::OUT_PAD, ACT, C::WAVES, C::NG,
                                  C::NCORR>),
                     dim3(blocks), dim3(64 * C::WAVES), lds, s, a, net, frags, biases, tab, sc,
                     step_a, list, counts, slot, pred);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || pred) return e;
  if (mid && (e = hipEventRecord(mid, s)) != hipSuccess) return e;
  // the rejected nodes are few and each takes the whole Heun pair: spread
  // them over many more threads than the step kernel's resident grid
  const unsigned fb_grid = (unsigned)(grid < 2048 ? 2048 : grid);
  hipLaunchKernelGGL(k_fallback<M>, dim3(fb_grid), dim3(256), 0, s, a, list, counts + slot,
                     step_a, total);
  return hipGetLastError();
}

template <class M>
static hipError_t sur_dispatch(const KArgs& a, const SurrogateNet& net, const __bf16* frags,
                               const float* biases, const float* tab, const SurrogateScales& sc,
                               int32_t step_a, int* list, int* counts, int slot, float* pred,
                               unsigned long long* total, hipEvent_t mid, int grid,
                               hipStream_t s) {
  if (net.act == FIB_ACT_RELU)
    return sur_launch<M, FIB_ACT_RELU>(a, net, frags, biases, tab, sc, step_a, list, counts, slot,
                                       pred, total, mid, grid, s);
  return sur_launch<M, FIB_ACT_SILU>(a, net, frags, biases, tab, sc, step_a, list, counts, slot,
                                     pred, total, mid, grid, s);
}

// Workgroups of k_midpoint<M, PRED, NCORR> resident at once on the current
// device (queried once per device and kernel; 0 if the query fails).
template <class M, int PRED>
static unsigned midpoint_resident_blocks() {
  static std::mutex mu;
  static unsigned cache[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  std::lock_guard<std::mutex> lock(mu);
  if (cache[dev] == 0) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, k_midpoint<M, PRED, SurCfg<M>::NCORR>, 256, 0) != hipSuccess ||
        cus <= 0 || per_cu <= 0)
      return 0;
    cache[dev] = (unsigned)cus * (unsigned)per_cu;
  }
  return cache[dev];
}

template <class M, int PRED>
static hipError_t pred_launch(const KArgs& a, const float* tab, int32_t step_a, int* list,
                              int* counts, int slot, unsigned long long* total, hipEvent_t mid,
                              int grid, hipStream_t s) {
  const int64_t need = (a.n_total + 255) / 256;
  const unsigned resident = midpoint_resident_blocks<M, PRED>();
  const int64_t cap = resident > 0 ? (int64_t)resident : need;
  const unsigned blocks = (unsigned)(need < cap ? need : cap);
  hipLaunchKernelGGL((k_midpoint<M, PRED, SurCfg<M>::NCORR>), dim3(blocks), dim3(256), 0, s, a,
                     tab, step_a, list, counts, slot);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (mid && (e = hipEventRecord(mid, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_fallback<M>, dim3((unsigned)grid), dim3(256), 0, s, a, list, counts + slot,
                     step_a, total);
  return hipGetLastError();
}

hipError_t launch_predictor_step(int model, int pred, const KArgs& a, const float* tab,
                                 int32_t step_a, int* list, int* counts, int slot,
                                 unsigned long long* total, int grid, hipEvent_t mid,
                                 hipStream_t s) {
  if (a.n_total == 0) return hipSuccess;
  if (model == 0)
    return pred == FIB_PRED_EULER
               ? pred_launch<SurHH, FIB_PRED_EULER>(a, tab, step_a, list, counts, slot, total, mid, grid, s)
               : pred_launch<SurHH, FIB_PRED_ZERO>(a, tab, step_a, list, counts, slot, total, mid, grid, s);
  return pred == FIB_PRED_EULER
             ? pred_launch<SurST57, FIB_PRED_EULER>(a, tab, step_a, list, counts, slot, total, mid, grid, s)
             : pred_launch<SurST57, FIB_PRED_ZERO>(a, tab, step_a, list, counts, slot, total, mid, grid, s);
}

size_t surrogate_lds_bytes(int model, const SurrogateNet& net) {
  return model == 0 ? sur_lds<SurHH>(net) : sur_lds<SurST57>(net);
}

hipError_t launch_surrogate_step(int model, const KArgs& a, const SurrogateNet& net,
                                 const __bf16* frags, const float* biases, const float* tab,
                                 const SurrogateScales& sc, int32_t step_a, int* list, int* counts,
                                 int slot, unsigned long long* total, int grid, hipEvent_t mid,
                                 hipStream_t s) {
  if (a.n_total == 0) return hipSuccess;
  if (model == 0)
    return sur_dispatch<SurHH>(a, net, frags, biases, tab, sc, step_a, list, counts, slot, nullptr,
                               total, mid, grid, s);
  return sur_dispatch<SurST57>(a, net, frags, biases, tab, sc, step_a, list, counts, slot, nullptr,
                               total, mid, grid, s);
}

hipError_t launch_surrogate_predict(int model, const KArgs& a, const SurrogateNet& net,
                                    const __bf16* frags, const float* biases, const float* tab,
                                    const SurrogateScales& sc, int32_t step_a, float* pred,
                                    int grid, hipStream_t s) {
  if (a.n_total == 0) return hipSuccess;
  if (model == 0)
    return sur_dispatch<SurHH>(a, net, frags, biases, tab, sc, step_a, nullptr, nullptr, 0, pred,
                               nullptr, nullptr, grid, s);
  return sur_dispatch<SurST57>(a, net, frags, biases, tab, sc, step_a, nullptr, nullptr, 0, pred,
                               nullptr, nullptr, grid, s);
}

}  // namespace fib
