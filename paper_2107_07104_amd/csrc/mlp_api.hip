// Host runtime of the surrogate network (C ABI in include/fib.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fib.h"
#include "mlp_internal.h"

namespace fib {
int set_error(int code, const char* msg);  // fib_api.hip
}

struct fib_mlp {
  fib::MlpShape shape{};
  hipStream_t stream = nullptr;
  int device = 0;             // device the network lives on
  float* d_params = nullptr;  // FP32 master parameters
  float* d_m = nullptr;       // Adam first moment
  float* d_v = nullptr;       // Adam second moment
  float* d_grad = nullptr;
  float* d_part = nullptr;    // per-chunk partial gradients
  float* d_loss_part = nullptr;
  int64_t part_chunks = 0;
  int64_t t = 0;              // Adam step count
};

// Scratch of fib_mlp_gradient_noalloc: the per-chunk partial gradients and
// losses, in a fixed array of every device's code object instead of memory
// allocated per call.  The array's name is a host-side stand-in: host code
// uses only the device address that hipGetSymbolAddress returns, looked up
// once per device with that device current (at fib_mlp_create) and kept in
// g_scratch below.  Every call on a device shares that device's array.
static constexpr int64_t kScratchFloats = (int64_t)1 << 22;  // 16 MiB per device
static __device__ __align__(256) float scratch[kScratchFloats];

namespace fib {
const MlpShape& mlp_shape(const fib_mlp* n) { return n->shape; }
const float* mlp_device_params(const fib_mlp* n) { return n->d_params; }
hipStream_t mlp_stream(const fib_mlp* n) { return n->stream; }
}  // namespace fib

namespace {

int mfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return fib::set_error(code, buf);
}

#define MHIP(expr)                                                                    \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return mfail(FIB_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch[kMaxDevices] = {};

// Looks up (once) the scratch address of `dev`, which must be current.
int scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return mfail(FIB_EUNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev]) return FIB_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return mfail(FIB_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  g_scratch[dev] = static_cast<float*>(p);
  return FIB_OK;
}

float* scratch_of(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch[dev];
}

int ensure_parts(fib_mlp* n, int64_t chunks) {
  if (chunks <= n->part_chunks) return FIB_OK;
  (void)hipStreamSynchronize(n->stream);
  (void)hipFree(n->d_part);
  (void)hipFree(n->d_loss_part);
  n->d_part = nullptr;
  n->d_loss_part = nullptr;
  n->part_chunks = 0;
  if (hipMalloc(&n->d_part, sizeof(float) * (size_t)chunks * n->shape.n_params) != hipSuccess ||
      hipMalloc(&n->d_loss_part, sizeof(float) * (size_t)chunks) != hipSuccess)
    return mfail(FIB_ENOMEM, "device allocation of %lld gradient chunks failed", (long long)chunks);
  n->part_chunks = chunks;
  return FIB_OK;
}

}  // namespace

extern "C" {

int fib_mlp_create(int32_t n_layers, const int32_t* sizes, int32_t activation, void* stream,
                   fib_mlp_t** out) {
  if (!out) return mfail(FIB_EINVAL, "null output pointer");
  *out = nullptr;
  if (n_layers < 1 || n_layers > fib::kMaxLayers || !sizes)
    return mfail(FIB_EINVAL, "the network needs 1..%d weight layers", fib::kMaxLayers);
  if (activation != FIB_ACT_SILU && activation != FIB_ACT_RELU)
    return mfail(FIB_EINVAL, "unknown activation %d", activation);
  fib::MlpShape s{};
  s.L = n_layers;
  s.act = activation;
  int64_t off = 0;
  for (int l = 0; l <= n_layers; ++l) {
    if (sizes[l] < 1 || sizes[l] > 512) return mfail(FIB_EINVAL, "layer width %d not in 1..512", sizes[l]);
    s.size[l] = sizes[l];
    s.pad[l] = (sizes[l] + fib::kPad - 1) / fib::kPad * fib::kPad;
  }
  for (int l = 1; l <= n_layers; ++l) {
    s.w_off[l] = (int)off;
    off += (int64_t)s.size[l] * s.size[l - 1];
    s.b_off[l] = (int)off;
    off += s.size[l];
  }
  s.n_params = (int)off;
  hipDeviceProp_t prop;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return mfail(FIB_EHIP, "no HIP device");
  if (fib::mlp_train_lds_bytes(s) > prop.sharedMemPerBlock)
    return mfail(FIB_EUNSUPPORTED, "network too wide for one workgroup's LDS");
  if (int rc = scratch_setup(dev)) return rc;
  fib_mlp* n = new (std::nothrow) fib_mlp();
  if (!n) return mfail(FIB_ENOMEM, "host allocation failed");
  n->shape = s;
  n->stream = (hipStream_t)stream;
  n->device = dev;
  const size_t bytes = sizeof(float) * (size_t)s.n_params;
  if (hipMalloc(&n->d_params, bytes) != hipSuccess || hipMalloc(&n->d_m, bytes) != hipSuccess ||
      hipMalloc(&n->d_v, bytes) != hipSuccess || hipMalloc(&n->d_grad, bytes) != hipSuccess) {
    fib_mlp_destroy(n);
    return mfail(FIB_ENOMEM, "device allocation failed");
  }
  if (hipMemset(n->d_params, 0, bytes) != hipSuccess || hipMemset(n->d_m, 0, bytes) != hipSuccess ||
      hipMemset(n->d_v, 0, bytes) != hipSuccess) {
    fib_mlp_destroy(n);
    return mfail(FIB_EHIP, "device initialization failed");
  }
  *out = n;
  return FIB_OK;
}

void fib_mlp_destroy(fib_mlp_t* n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->stream);
  (void)hipFree(n->d_params);
  (void)hipFree(n->d_m);
  (void)hipFree(n->d_v);
  (void)hipFree(n->d_grad);
  (void)hipFree(n->d_part);
  (void)hipFree(n->d_loss_part);
  delete n;
}

int64_t fib_mlp_n_params(const fib_mlp_t* n) { return n ? n->shape.n_params : 0; }

int fib_mlp_set_params(fib_mlp_t* n, const float* params, int64_t count) {
  if (!n || !params) return mfail(FIB_EINVAL, "null argument");
  if (count != n->shape.n_params) return mfail(FIB_EINVAL, "expected %d parameters", n->shape.n_params);
  MHIP(hipMemcpyAsync(n->d_params, params, sizeof(float) * count, hipMemcpyHostToDevice, n->stream));
  MHIP(hipStreamSynchronize(n->stream));
  return FIB_OK;
}

int fib_mlp_get_params(fib_mlp_t* n, float* params, int64_t count) {
  if (!n || !params) return mfail(FIB_EINVAL, "null argument");
  if (count != n->shape.n_params) return mfail(FIB_EINVAL, "expected %d parameters", n->shape.n_params);
  MHIP(hipMemcpyAsync(params, n->d_params, sizeof(float) * count, hipMemcpyDeviceToHost, n->stream));
  MHIP(hipStreamSynchronize(n->stream));
  return FIB_OK;
}

int fib_mlp_forward(fib_mlp_t* n, const float* X, int64_t B, float* O) {
  if (!n || B < 0 || (B > 0 && (!X || !O))) return mfail(FIB_EINVAL, "bad arguments");
  MHIP(fib::launch_mlp_forward(n->shape, n->d_params, X, B, O, n->stream));
  return FIB_OK;
}

int fib_mlp_gradient(fib_mlp_t* n, const float* X, const float* T, int64_t B, float* grad,
                     float* loss) {
  if (!n || B < 1 || !X || !T) return mfail(FIB_EINVAL, "bad arguments");
  const int64_t chunks = (B + fib::kChunk - 1) / fib::kChunk;
  if (int rc = ensure_parts(n, chunks)) return rc;
  MHIP(fib::launch_mlp_grad(n->shape, n->d_params, X, T, B, n->d_part, n->d_loss_part,
                            grad ? grad : n->d_grad, loss, n->stream));
  return FIB_OK;
}

int fib_mlp_gradient_noalloc(fib_mlp_t* n, const float* X, const float* T, int64_t B,
                             float* grad, float* loss) {
  if (!n || B < 1 || !X || !T) return mfail(FIB_EINVAL, "bad arguments");
  const int64_t chunks = (B + fib::kChunk - 1) / fib::kChunk;
  const int64_t need = chunks * (int64_t)n->shape.n_params + chunks;
  if (need > kScratchFloats)
    return mfail(FIB_EINVAL, "batch of %lld samples needs %lld scratch floats, more than the "
                 "%lld this entry point holds (at most %lld samples for this network)",
                 (long long)B, (long long)need, (long long)kScratchFloats,
                 (long long)(kScratchFloats / (n->shape.n_params + 1) * fib::kChunk));
  float* base = scratch_of(n->device);
  if (!base) return mfail(FIB_ESTATE, "scratch of device %d not set up", n->device);
  float* part = base;
  float* loss_part = base + chunks * (int64_t)n->shape.n_params;
  MHIP(fib::launch_mlp_grad(n->shape, n->d_params, X, T, B, part, loss_part,
                            grad ? grad : n->d_grad, loss, n->stream));
  return FIB_OK;
}

int fib_column_stats(const float* A, int64_t rows, int32_t cols, void* stream, double* mean,
                     double* std, float* cmin, float* cmax) {
  if (!A || rows < 1 || cols < 1 || cols > 64 || !mean || !std || !cmin || !cmax)
    return mfail(FIB_EINVAL, "bad arguments (1 <= cols <= 64, rows >= 1)");
  hipStream_t st = (hipStream_t)stream;
  const int blocks = (int)std::min<int64_t>(1024, (rows + 255) / 256);
  double* d = nullptr;
  float* f = nullptr;
  const size_t nd = (size_t)blocks * cols + 3 * (size_t)cols, nf = 2 * ((size_t)blocks + 1) * cols;
  if (hipMalloc(&d, sizeof(double) * nd) != hipSuccess || hipMalloc(&f, sizeof(float) * nf) != hipSuccess) {
    (void)hipFree(d);
    return mfail(FIB_ENOMEM, "device allocation failed");
  }
  double *part = d, *sum = part + (size_t)blocks * cols, *mu = sum + cols, *sq = mu + cols;
  float *pmin = f, *pmax = pmin + (size_t)blocks * cols, *lo = pmax + (size_t)blocks * cols,
        *hi = lo + cols;
  std::vector<double> hsum(cols), hsq(cols);
  int rc = FIB_OK;
  hipError_t e = fib::launch_col_stats(A, rows, cols, part, pmin, pmax, blocks, sum, lo, hi,
                                       nullptr, nullptr, st);
  if (e == hipSuccess) e = hipMemcpyAsync(hsum.data(), sum, sizeof(double) * cols, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) {
    for (int k = 0; k < cols; ++k) mean[k] = hsum[k] / (double)rows;
    e = hipMemcpyAsync(mu, mean, sizeof(double) * cols, hipMemcpyHostToDevice, st);
  }
  if (e == hipSuccess)
    e = fib::launch_col_stats(A, rows, cols, part, pmin, pmax, blocks, sum, lo, hi, mu, sq, st);
  if (e == hipSuccess) e = hipMemcpyAsync(hsq.data(), sq, sizeof(double) * cols, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(cmin, lo, sizeof(float) * cols, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(cmax, hi, sizeof(float) * cols, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) {
    for (int k = 0; k < cols; ++k) std[k] = rows > 1 ? std::sqrt(hsq[k] / (double)(rows - 1)) : 0.0;
  } else {
    rc = mfail(FIB_EHIP, "column statistics: %s", hipGetErrorString(e));
  }
  (void)hipFree(d);
  (void)hipFree(f);
  return rc;
}

int fib_normalize_rows(const float* A, int64_t rows, int32_t cols, const float* shift,
                       const float* scale, double extra, float* Y, int32_t ldy, void* stream) {
  if (!A || !Y || !shift || !scale || rows < 0 || cols < 1 || cols > 64 || ldy < cols)
    return mfail(FIB_EINVAL, "bad arguments (1 <= cols <= 64, ldy >= cols)");
  if (rows == 0) return FIB_OK;
  hipStream_t st = (hipStream_t)stream;
  float* d = nullptr;
  if (hipMalloc(&d, sizeof(float) * 2 * cols) != hipSuccess)
    return mfail(FIB_ENOMEM, "device allocation failed");
  hipError_t e = hipMemcpyAsync(d, shift, sizeof(float) * cols, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d + cols, scale, sizeof(float) * cols, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = fib::launch_normalize(A, rows, cols, d, d + cols, (float)extra, Y, ldy, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d);
  if (e != hipSuccess) return mfail(FIB_EHIP, "normalize: %s", hipGetErrorString(e));
  return FIB_OK;
}

int fib_mlp_adam_step(fib_mlp_t* n, const float* X, const float* T, int64_t B, double lr,
                      float* loss) {
  if (!n || B < 1 || !X || !T || !(lr > 0.0)) return mfail(FIB_EINVAL, "bad arguments");
  const int64_t chunks = (B + fib::kChunk - 1) / fib::kChunk;
  if (int rc = ensure_parts(n, chunks)) return rc;
  MHIP(fib::launch_mlp_grad(n->shape, n->d_params, X, T, B, n->d_part, n->d_loss_part, n->d_grad,
                            loss, n->stream));
  n->t += 1;
  MHIP(fib::launch_mlp_adam(n->d_params, n->d_m, n->d_v, n->d_grad, n->shape.n_params, (float)lr,
                            0.9f, 0.999f, 1e-8f, n->t, n->stream));
  return FIB_OK;
}

int fib_mlp_reset_optimizer(fib_mlp_t* n) {
  if (!n) return mfail(FIB_EINVAL, "null network");
  const size_t bytes = sizeof(float) * (size_t)n->shape.n_params;
  MHIP(hipMemsetAsync(n->d_m, 0, bytes, n->stream));
  MHIP(hipMemsetAsync(n->d_v, 0, bytes, n->stream));
  n->t = 0;
  return FIB_OK;
}

}  // extern "C"
