// Internal description of the surrogate step: the packed network and the
// per-state scalings.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fib_internal.h"

namespace fib {

constexpr int kSurMaxLayers = 6;
constexpr int kSurMaxStates = 64;

// Network packed for the matrix cores.  Layer l = 1..L maps n_in[l] to
// n_out[l] features; its weights are pad_out[l]/16 x pad_in[l]/32
// fragments of 64 lanes x 8 BF16 (512 elements), fragment (ob, kb) at
// index frag_off[l] + ob * (pad_in[l]/32) + kb; its biases (padded to
// pad_out[l]) start at bias_off[l].  w_off / b_off locate the layer in the
// flat FP32 parameters.  act: hidden activation (FIB_ACT_*).
struct SurrogateNet {
  int L;
  int act;
  int n_in[kSurMaxLayers + 2], n_out[kSurMaxLayers + 2];
  int pad_in[kSurMaxLayers + 2], pad_out[kSurMaxLayers + 2];
  int w_off[kSurMaxLayers + 2], b_off[kSurMaxLayers + 2];
  int frag_off[kSurMaxLayers + 2];
  int bias_off[kSurMaxLayers + 2];
  int64_t frag_elems;
  int bias_elems;
};

// Per-state tables of the surrogate step (device memory, kSurTabFloats
// floats), laid out so one LDS read serves a state in each use:
//   kTabIn,  float2: (in_scale_k, -in_shift_k in_scale_k), so the input is
//            x_k = u_k in_scale_k - in_shift_k in_scale_k;
//   kTabMid, float2: (out_scale_k / 2, out_shift_k / 2 + rest_k), so the
//            midpoint is y_k = rest_k + u_k + du_k / 2 with
//            du_k = out_shift_k + out_scale_k o_k;
//   kTabChk, float4: (out_scale_k, out_shift_k, tol res_k, rest_k): the
//            prediction, the absolute acceptance threshold and the resting
//            state the offsets u are taken from.
constexpr int kTabIn = 0;
constexpr int kTabMid = 2 * kSurMaxStates;
constexpr int kTabChk = 4 * kSurMaxStates;
constexpr int kSurTabFloats = 8 * kSurMaxStates;

// Scalars of the step: network inputs (n_states, or n_states + 1 with the
// stimulus flag I * flag_scale) and the acceptance tolerance.
struct SurrogateScales {
  int n_in;
  float flag_scale;
  float tol;
};

hipError_t launch_pack(const SurrogateNet& net, const float* params, __bf16* frags, float* biases,
                       hipStream_t s);
size_t surrogate_lds_bytes(int model, const SurrogateNet& net);
// One surrogate step: appends rejected nodes to list through counts[slot]
// and clears counts[slot ^ 1] for the next step (the caller alternates the
// slot between launches; both counters start at zero).
// The fallback kernel adds each step's rejection count to *total (nullable);
// `mid` (nullable) is recorded between the step kernel and the fallback.
hipError_t launch_surrogate_step(int model, const KArgs& a, const SurrogateNet& net,
                                 const __bf16* frags, const float* biases, const float* tab,
                                 const SurrogateScales& sc, int32_t step_a, int* list, int* counts,
                                 int slot, unsigned long long* total, int grid, hipEvent_t mid,
                                 hipStream_t s);
// The same step with a closed-form predictor (FIB_PRED_ZERO or
// FIB_PRED_EULER) instead of the network; tab as for the network step (only
// its kTabChk thresholds and resting state are read).
hipError_t launch_predictor_step(int model, int pred, const KArgs& a, const float* tab,
                                 int32_t step_a, int* list, int* counts, int slot,
                                 unsigned long long* total, int grid, hipEvent_t mid,
                                 hipStream_t s);
hipError_t launch_surrogate_predict(int model, const KArgs& a, const SurrogateNet& net,
                                    const __bf16* frags, const float* biases, const float* tab,
                                    const SurrogateScales& sc, int32_t step_a, float* pred,
                                    int grid, hipStream_t s);

}  // namespace fib
