// Surrogate split-step kernels (gfx950).
//
// In surrogate mode the split schedule replaces the pair of reaction halves
// that meet between two diffusion steps, R(dt/2) of step n followed by
// R(dt/2) of step n+1, by one implicit-midpoint step of width dt,
//   du* = dt G(y + du*/2, I),
// solved by fixed-point iteration from the network's prediction du:
//   du1 = dt G(y + du/2, I),   du2 = dt G(y + du1/2, I).
// The iteration contracts by q = dt |dG/dy| / 2 (a few percent at the
// split steps used here), so |du1 - du| measures the network's error and
// du2 lies within about q^2 |du1 - du| of du*.  A node keeps du2 only if
// |du1 - du|_k <= tol * atol_k for every state k; every other node -- and
// every node whose stimulus changes between the two halves -- is appended
// to a compacted list that the fallback kernel advances with the plain
// Heun substeps.  The state at the end of step n, which the pair never
// forms, is taken as the midpoint y + du2/2 for the activation-time
// observable; steps that write V_m samples run the plain path everywhere.
//
// Network on the matrix cores, one wave per 64 nodes: nodes are the N
// dimension of v_mfma_f32_16x16x32_bf16 (16 nodes per instruction, four
// groups per wave) and the weights are the A operand, pre-packed in BF16
// fragments that the workgroup stages in LDS.  A layer's output D holds, in
// lane l, features 16 ob + 4 (l / 16) + j of node l % 16; the next layer
// takes its K-block kb from the output blocks 2 kb and 2 kb + 1 of the same
// lane, so activations stay in registers and the weight packing absorbs the
// implied permutation of the K index:
//   K index 8 g + i  <->  feature 32 kb + 4 g + i          (i < 4)
//                          feature 32 kb + 16 + 4 g + i - 4 (i >= 4).
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

__device__ __forceinline__ float silu_fast(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

// Model adapters: number of states, offsets -> increments of one Heun step.
struct SurHH {
  static constexpr int S = 4;
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
  __device__ static void rhs(const float (&u)[S], const float* ref, float I, float inv_cm,
                             float (&d)[S]) {
    st57::rhs<float>(u, ref, I, inv_cm, d);
  }
  __device__ static void heun(float (&u)[S], const float* ref, float I, float tau, float inv_cm) {
    st57::heun(u, ref, I, tau, inv_cm);
  }
};

// Observables at the end of split step `step` from V offset v1 (see
// k_react in fib_kernels.hip for the same rules).
__device__ __forceinline__ void observe(const KArgs& A, int64_t i, int32_t step, float v1) {
  const float v0 = A.v_prev[i];
  const float uth = A.v_th - A.rest[0];
  if (isinf(A.t_act[i]) && v0 < uth && v1 >= uth)
    A.t_act[i] = fmaf(A.dt, (uth - v0) / (v1 - v0), (float)step * A.dt);
  A.v_prev[i] = v1;
  if (!isfinite(v1)) atomicOr(A.flag, 1);
}

// One wave of 64 nodes through the network.  X: LDS staging [64][KIN_PAD]
// (BF16, node-major); O: LDS staging [64][OUT_PAD] (FP32).  The packed
// weights and biases are in LDS (wfr, wb).
template <int KIN_PAD, int H, int NHID, int OUT_PAD>
__device__ __forceinline__ void wave_network(const __bf16* X, float* O, const __bf16* wfr,
                                             const float* wb, const SurrogateNet& net,
                                             int lane) {
  constexpr int HB = H / 16;         // output blocks of a hidden layer
  constexpr int KB0 = KIN_PAD / 32;  // K-blocks of the input layer
  constexpr int KBH = H / 32;        // K-blocks of a hidden-to-next layer
  constexpr int OB = OUT_PAD / 16;   // output blocks of the last layer
  const int r = lane & 15, g = lane >> 4;
  const v8bf* frag = reinterpret_cast<const v8bf*>(wfr);
  for (int grp = 0; grp < 4; ++grp) {
    const int node = 16 * grp + r;
    // input layer
    v8bf b0[KB0];
#pragma unroll
    for (int kb = 0; kb < KB0; ++kb)
      b0[kb] = *reinterpret_cast<const v8bf*>(X + node * KIN_PAD + 32 * kb + 8 * g);
    v4f acc[HB];
#pragma unroll
    for (int ob = 0; ob < HB; ++ob) {
      v4f c = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kb = 0; kb < KB0; ++kb)
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag[(net.frag_off[1] + ob * KB0 + kb) * 64 + lane],
                                                    b0[kb], c, 0, 0, 0);
      acc[ob] = c;
    }
    // hidden layers 2..NHID (hidden to hidden), then the output layer
    int layer = 1;
#pragma unroll
    for (int hl = 0; hl < NHID; ++hl, ++layer) {
      // bias + SiLU, pack to the next layer's B operands
      v8bf b[KBH];
#pragma unroll
      for (int ob = 0; ob < HB; ++ob) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float z = acc[ob][j] + wb[net.bias_off[layer] + 16 * ob + 4 * g + j];
          b[ob >> 1][(ob & 1) * 4 + j] = (__bf16)silu_fast(z);
        }
      }
      if (hl + 1 < NHID) {
#pragma unroll
        for (int ob = 0; ob < HB; ++ob) {
          v4f c = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int kb = 0; kb < KBH; ++kb)
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                frag[(net.frag_off[layer + 1] + ob * KBH + kb) * 64 + lane], b[kb], c, 0, 0, 0);
          acc[ob] = c;
        }
      } else {
        // output layer
#pragma unroll
        for (int ob = 0; ob < OB; ++ob) {
          v4f c = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int kb = 0; kb < KBH; ++kb)
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                frag[(net.frag_off[layer + 1] + ob * KBH + kb) * 64 + lane], b[kb], c, 0, 0, 0);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int f = 16 * ob + 4 * g + j;
            O[node * OUT_PAD + f] = c[j] + wb[net.bias_off[layer + 1] + f];
          }
        }
      }
    }
  }
}

// Staging of one wave in LDS: the FP32 network outputs O [64][OUT_PAD] and,
// aliased into the same region, the BF16 inputs X [64][KIN_PAD] at byte
// offset XOFF.  Group g (nodes 16 g .. 16 g + 15) reads its X rows before
// it writes its O rows, and its O rows never reach the X rows of a later
// group.
template <int KIN_PAD, int OUT_PAD>
struct Staging {
  static constexpr int kOBytes = 64 * OUT_PAD * 4;
  static constexpr int kXBytes = 64 * KIN_PAD * 2;
  static constexpr int kGap = 3 * 16 * (OUT_PAD * 4 - KIN_PAD * 2);
  static constexpr int kXOff = kGap > 0 ? (kGap + 15) / 16 * 16 : 0;
  static constexpr int kBytes = (kOBytes > kXOff + kXBytes ? kOBytes : kXOff + kXBytes);
};

// Surrogate reaction pair for every node: finishes step `step_a` and
// starts step `step_a + 1`.  Rejected nodes are appended to list[] through
// count[0] (one atomic per wave).  With `pred` set, the kernel only writes
// the predicted increments du ([S][n_total]) and changes no state.
// Persistent: each wave walks the 64-node tiles tile = wave_id,
// wave_id + waves, ...  Launch: 256 threads.
template <class M, int KIN_PAD, int H, int NHID, int OUT_PAD>
__global__ __launch_bounds__(256) void k_surrogate(KArgs A, SurrogateNet net,
                                                   const __bf16* __restrict__ frags,
                                                   const float* __restrict__ biases,
                                                   SurrogateScales sc, int32_t step_a,
                                                   int* __restrict__ list,
                                                   int* __restrict__ count,
                                                   float* __restrict__ pred) {
  extern __shared__ float lds_f[];
  using St = Staging<KIN_PAD, OUT_PAD>;
  constexpr int S = M::S;
  __bf16* wfr = reinterpret_cast<__bf16*>(lds_f);
  float* wb = lds_f + net.frag_elems / 2;
  char* stage = reinterpret_cast<char*>(wb + net.bias_elems);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float* O = reinterpret_cast<float*>(stage + wave * St::kBytes);
  __bf16* X = reinterpret_cast<__bf16*>(stage + wave * St::kBytes + St::kXOff);

  {
    const uint4* src = reinterpret_cast<const uint4*>(frags);
    uint4* dst = reinterpret_cast<uint4*>(wfr);
    for (int e = threadIdx.x; e < net.frag_elems / 8; e += 256) dst[e] = src[e];
    for (int e = threadIdx.x; e < net.bias_elems; e += 256) wb[e] = biases[e];
  }
  __syncthreads();

  const int64_t nt = A.n_total;
  const int64_t tiles = (nt + 63) / 64;
  const int32_t step_b = step_a + 1;
  const float span = 2.0f * A.tau * (float)A.n_sub;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < tiles;
       tile += (int64_t)gridDim.x * 4) {
    const int64_t i = tile * 64 + lane;
    const bool real = i < nt;
    float Ia = 0.0f, Ib = 0.0f;
    if (real) {
      const uint32_t sid = (uint32_t)A.node_stim[i];
      Ia = stim_current(sid, A.stim, step_a);
      Ib = stim_current(sid, A.stim, step_b);
    }
    // network inputs of this lane's node
#pragma unroll
    for (int k = 0; k < KIN_PAD; ++k) {
      float x = 0.0f;
      if (k < S && k < sc.n_in) {
        const float u = real ? A.state[k * nt + i] : 0.0f;
        x = (u - sc.in_shift[k]) * sc.in_scale[k];
      } else if (k == S && k < sc.n_in) {
        x = Ia * sc.flag_scale;
      }
      X[lane * KIN_PAD + k] = (__bf16)x;
    }
    wave_network<KIN_PAD, H, NHID, OUT_PAD>(X, O, wfr, wb, net, lane);
    if (pred) {
      if (real) {
#pragma unroll
        for (int k = 0; k < S; ++k)
          pred[k * nt + i] = fmaf(O[lane * OUT_PAD + k], sc.out_scale[k], sc.out_shift[k]);
      }
      continue;
    }

    // residual of the prediction at the midpoint y + du / 2
    bool ok = false;
    if (real) {
      float ym[S], G[S];
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const float du = fmaf(O[lane * OUT_PAD + k], sc.out_scale[k], sc.out_shift[k]);
        ym[k] = fmaf(0.5f, du, A.state[k * nt + i]);
      }
      M::rhs(ym, A.rest, Ia, A.inv_cm, G);
      // a comparison with NaN is false: a non-finite prediction is rejected
      bool within = true;
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const float du = fmaf(O[lane * OUT_PAD + k], sc.out_scale[k], sc.out_shift[k]);
        const float du1 = span * G[k];
        within &= fabsf(du1 - du) * sc.inv_res[k] <= sc.tol;
        ym[k] = fmaf(0.5f * span, G[k], A.state[k * nt + i]);
      }
      const bool flag_ok = sc.n_in > S || Ia == 0.0f;
      ok = within && flag_ok && Ia == Ib;
      if (ok) {
        M::rhs(ym, A.rest, Ia, A.inv_cm, G);
        const float u0 = A.state[i];
        observe(A, i, step_a, fmaf(0.5f * span, G[0], u0));
#pragma unroll
        for (int k = 0; k < S; ++k) A.state[k * nt + i] = fmaf(span, G[k], A.state[k * nt + i]);
      }
    }
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

// Plain reaction pair (second half of step_a, observables, first half of
// step_a + 1) for the nodes in list[0..count).  Grid-stride loop, so the
// grid does not depend on the count.
template <class M>
__global__ __launch_bounds__(256) void k_fallback(KArgs A, const int* __restrict__ list,
                                                  const int* __restrict__ count, int32_t step_a) {
  constexpr int S = M::S;
  const int n = *count;
  const int64_t nt = A.n_total;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    const int64_t i = list[e];
    float u[S];
#pragma unroll
    for (int k = 0; k < S; ++k) u[k] = A.state[k * nt + i];
    const uint32_t sid = (uint32_t)A.node_stim[i];
    const float Ia = stim_current(sid, A.stim, step_a);
    for (int s = 0; s < A.n_sub; ++s) M::heun(u, A.rest, Ia, A.tau, A.inv_cm);
    observe(A, i, step_a, u[0]);
    const float Ib = stim_current(sid, A.stim, step_a + 1);
    for (int s = 0; s < A.n_sub; ++s) M::heun(u, A.rest, Ib, A.tau, A.inv_cm);
#pragma unroll
    for (int k = 0; k < S; ++k) A.state[k * nt + i] = u[k];
  }
}

__global__ void k_zero_int(int* p) { *p = 0; }

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

template <class M, int KIN_PAD, int H, int NHID, int OUT_PAD>
static size_t sur_lds(const SurrogateNet& net) {
  return (size_t)net.frag_elems * 2 + (size_t)net.bias_elems * 4 +
         (size_t)4 * Staging<KIN_PAD, OUT_PAD>::kBytes;
}

template <class M, int KIN_PAD, int H, int NHID, int OUT_PAD>
static hipError_t sur_step(const KArgs& a, const SurrogateNet& net, const __bf16* frags,
                           const float* biases, const SurrogateScales& sc, int32_t step_a,
                           int* list, int* count, int grid, hipStream_t s) {
  const size_t lds = sur_lds<M, KIN_PAD, H, NHID, OUT_PAD>(net);
  const int64_t tiles = (a.n_total + 63) / 64;
  const int64_t need = (tiles + 3) / 4;
  const unsigned blocks = (unsigned)(need < grid ? need : grid);
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, count);
  hipLaunchKernelGGL((k_surrogate<M, KIN_PAD, H, NHID, OUT_PAD>), dim3(blocks), dim3(256), lds, s,
                     a, net, frags, biases, sc, step_a, list, count, nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fallback<M>, dim3((unsigned)grid), dim3(256), 0, s, a, list, count, step_a);
  return hipGetLastError();
}

template <class M, int KIN_PAD, int H, int NHID, int OUT_PAD>
static hipError_t sur_predict(const KArgs& a, const SurrogateNet& net, const __bf16* frags,
                              const float* biases, const SurrogateScales& sc, int32_t step_a,
                              float* pred, int grid, hipStream_t s) {
  const size_t lds = sur_lds<M, KIN_PAD, H, NHID, OUT_PAD>(net);
  const int64_t tiles = (a.n_total + 63) / 64;
  const int64_t need = (tiles + 3) / 4;
  const unsigned blocks = (unsigned)(need < grid ? need : grid);
  hipLaunchKernelGGL((k_surrogate<M, KIN_PAD, H, NHID, OUT_PAD>), dim3(blocks), dim3(256), lds, s,
                     a, net, frags, biases, sc, step_a, nullptr, nullptr, pred);
  return hipGetLastError();
}

size_t surrogate_lds_bytes(int model, const SurrogateNet& net) {
  if (model == 0) return sur_lds<SurHH, 32, 64, 3, 16>(net);
  return sur_lds<SurST57, 64, 128, 2, 64>(net);
}

hipError_t launch_surrogate_step(int model, const KArgs& a, const SurrogateNet& net,
                                 const __bf16* frags, const float* biases,
                                 const SurrogateScales& sc, int32_t step_a, int* list, int* count,
                                 int grid, hipStream_t s) {
  if (a.n_total == 0) return hipSuccess;
  if (model == 0)  // 5 -> 64 -> 64 -> 64 -> 4
    return sur_step<SurHH, 32, 64, 3, 16>(a, net, frags, biases, sc, step_a, list, count, grid, s);
  // 57 -> 128 -> 128 -> 57
  return sur_step<SurST57, 64, 128, 2, 64>(a, net, frags, biases, sc, step_a, list, count, grid, s);
}

hipError_t launch_surrogate_predict(int model, const KArgs& a, const SurrogateNet& net,
                                    const __bf16* frags, const float* biases,
                                    const SurrogateScales& sc, int32_t step_a, float* pred,
                                    int grid, hipStream_t s) {
  if (a.n_total == 0) return hipSuccess;
  if (model == 0)
    return sur_predict<SurHH, 32, 64, 3, 16>(a, net, frags, biases, sc, step_a, pred, grid, s);
  return sur_predict<SurST57, 64, 128, 2, 64>(a, net, frags, biases, sc, step_a, pred, grid, s);
}

}  // namespace fib
