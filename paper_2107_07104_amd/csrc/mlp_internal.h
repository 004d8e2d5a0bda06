// Internal shape description of the surrogate network, shared by the host
// runtime and the network kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fib {

constexpr int kMaxLayers = 6;  // weight layers
constexpr int kChunk = 32;     // samples per training workgroup
constexpr int kPad = 32;       // feature dimensions are padded to multiples of this

// Flat parameter layout (FP32): for every layer l = 1..L the weight matrix
// W_l (size[l] x size[l-1], row-major) followed by the bias b_l.
struct MlpShape {
  int L;                        // number of weight layers
  int size[kMaxLayers + 1];     // features per layer, size[0] = inputs
  int pad[kMaxLayers + 1];      // size rounded up to kPad
  int w_off[kMaxLayers + 1];    // offset of W_l in the flat parameters
  int b_off[kMaxLayers + 1];    // offset of b_l
  int n_params;
  int act;                      // hidden activation: FIB_ACT_SILU or FIB_ACT_RELU
};

size_t mlp_train_lds_bytes(const MlpShape& s);
hipError_t launch_mlp_forward(const MlpShape& s, const float* params, const float* X, int64_t B,
                              float* O, hipStream_t st);
hipError_t launch_mlp_grad(const MlpShape& s, const float* params, const float* X, const float* T,
                           int64_t B, float* part, float* loss_part, float* grad, float* loss,
                           hipStream_t st);
hipError_t launch_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t n, float lr,
                           float b1, float b2, float eps, int64_t t, hipStream_t st);
// Column sums, minima and maxima of A (rows x cols, cols <= 64) into
// device arrays sum/cmin/cmax; with `mean` (device) also the sums of
// squared deviations into sq.  part/pmin/pmax hold blocks x cols.
hipError_t launch_col_stats(const float* A, int64_t rows, int cols, double* part, float* pmin,
                            float* pmax, int blocks, double* sum, float* cmin, float* cmax,
                            const double* mean, double* sq, hipStream_t st);
// Y[r][k] = (A[r][k] - shift[k]) scale[k]; Y[r][cols] = extra if ldy > cols.
hipError_t launch_normalize(const float* A, int64_t rows, int cols, const float* shift,
                            const float* scale, float extra, float* Y, int ldy, hipStream_t st);

}  // namespace fib

struct fib_mlp;
namespace fib {
// Shape and device parameters of a network object (mlp_api.hip).
const MlpShape& mlp_shape(const fib_mlp* n);
const float* mlp_device_params(const fib_mlp* n);
hipStream_t mlp_stream(const fib_mlp* n);

}  // namespace fib
