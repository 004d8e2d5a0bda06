// Surrogate network kernels (gfx950): batched forward pass, backpropagation
// and Adam for a multilayer perceptron with SiLU or ReLU hidden layers and
// a linear output, trained on the mean squared error.  Every matrix product runs on
// the matrix cores (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32
// accumulation); the master weights, moments and gradients are FP32.
//
// Operand layout of v_mfma_f32_16x16x32_bf16 on a 64-lane wave (checked on
// the device): lane l supplies A[l % 16][8 (l / 16) + i] and
// B[8 (l / 16) + i][l % 16] for i = 0..7, and receives
// D[4 (l / 16) + j][l % 16] for j = 0..3.
//
// Training is a one-time cost next to the solver, so these kernels favour a
// plain structure: one wave per workgroup, a chunk of kChunk samples, every
// activation in LDS in FP32, operands converted to BF16 when they are
// loaded into the matrix-core registers.
#include "../../include/fib.h"
#include "fib_internal.h"
#include "mlp_internal.h"

namespace fib {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Read-only view of a matrix with strides and a zero border:
// (i, j) -> p[i * s0 + j * s1] when i < n0 and j < n1, else 0.
struct MatRef {
  const float* p;
  int s0, s1, n0, n1;
  __device__ float at(int i, int j) const {
    return (i < n0 && j < n1) ? p[(int64_t)i * s0 + (int64_t)j * s1] : 0.0f;
  }
};

// C (M x N) = A (M x K) * B (K x N) on one wave; M, N multiples of 16, K a
// multiple of 32.  C(i, j) is written to c[i * sc0 + j * sc1] for i < cm,
// j < cn (the rest of the padded block is dropped).
__device__ void wave_gemm(const MatRef& A, const MatRef& B, float* c, int sc0, int sc1, int cm,
                          int cn, int M, int N, int K, int lane) {
  const int r = lane & 15, g = lane >> 4;
  for (int mb = 0; mb < M; mb += 16) {
    for (int nb = 0; nb < N; nb += 16) {
      v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
      for (int kb = 0; kb < K; kb += 32) {
        v8bf a, b;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          a[i] = (__bf16)A.at(mb + r, kb + 8 * g + i);
          b[i] = (__bf16)B.at(kb + 8 * g + i, nb + r);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = mb + 4 * g + j, jj = nb + r;
        if (i < cm && jj < cn) c[(int64_t)i * sc0 + (int64_t)jj * sc1] = acc[j];
      }
    }
  }
}

__device__ __forceinline__ float silu(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_grad(float z) {
  const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
  return s * fmaf(z, 1.0f - s, 1.0f);
}
// Hidden activation and its derivative (ReLU'(0) taken as 0).
__device__ __forceinline__ float act_fn(int act, float z) {
  return act == FIB_ACT_RELU ? fmaxf(z, 0.0f) : silu(z);
}
__device__ __forceinline__ float act_grad(int act, float z) {
  return act == FIB_ACT_RELU ? (z > 0.0f ? 1.0f : 0.0f) : silu_grad(z);
}

// LDS plan of the training kernel (floats): for every layer l = 0..L an
// activation block act_l [kChunk x pad(n_l)], for every hidden layer a
// pre-activation block z_l, and two gradient blocks [kChunk x pad(max n)].
struct TrainLds {
  int act[kMaxLayers + 1];
  int z[kMaxLayers + 1];
  int dz[2];
  int total;
};

__host__ __device__ inline TrainLds train_lds(const MlpShape& s) {
  TrainLds t{};
  int o = 0;
  int pmax = 0;
  for (int l = 0; l <= s.L; ++l) {
    t.act[l] = o;
    o += kChunk * s.pad[l];
    pmax = s.pad[l] > pmax ? s.pad[l] : pmax;
  }
  for (int l = 1; l < s.L; ++l) {
    t.z[l] = o;
    o += kChunk * s.pad[l];
  }
  t.dz[0] = o;
  o += kChunk * pmax;
  t.dz[1] = o;
  o += kChunk * pmax;
  t.total = o;
  return t;
}

size_t mlp_train_lds_bytes(const MlpShape& s) { return sizeof(float) * (size_t)train_lds(s).total; }

// Forward pass of one chunk of samples into LDS (activations, and the
// pre-activations of hidden layers when keep_z).
__device__ void chunk_forward(const MlpShape& s, const float* __restrict__ params,
                              const float* __restrict__ X, int64_t B, int64_t s0, float* lds,
                              const TrainLds& t, bool keep_z, int lane) {
  // inputs, zero padded
  const int n0 = s.size[0], p0 = s.pad[0];
  for (int e = lane; e < kChunk * p0; e += 64) {
    const int i = e / p0, j = e % p0;
    const int64_t row = s0 + i;
    lds[t.act[0] + e] = (row < B && j < n0) ? X[row * n0 + j] : 0.0f;
  }
  __syncthreads();
  for (int l = 1; l <= s.L; ++l) {
    const int nin = s.size[l - 1], nout = s.size[l];
    const float* W = params + s.w_off[l];
    const float* bias = params + s.b_off[l];
    // z = act_{l-1} W^T  (chunk x out)
    const MatRef A{lds + t.act[l - 1], s.pad[l - 1], 1, kChunk, s.pad[l - 1]};
    const MatRef Bw{W, 1, nin, nin, nout};  // (k = in, n = out) -> W[out][in]
    float* dst = lds + (l < s.L && keep_z ? t.z[l] : t.act[l]);
    wave_gemm(A, Bw, dst, s.pad[l], 1, kChunk, s.pad[l], kChunk, s.pad[l], s.pad[l - 1], lane);
    __syncthreads();
    for (int e = lane; e < kChunk * s.pad[l]; e += 64) {
      const int j = e % s.pad[l];
      float v = j < nout ? dst[e] + bias[j] : 0.0f;
      if (l < s.L) {
        if (keep_z) dst[e] = v;
        v = j < nout ? act_fn(s.act, v) : 0.0f;
      }
      lds[t.act[l] + e] = v;
    }
    __syncthreads();
  }
}

// Batched forward pass: O[b][k] for b < B.  One wave per chunk of samples.
__global__ __launch_bounds__(64) void k_mlp_forward(MlpShape s, const float* __restrict__ params,
                                                    const float* __restrict__ X, int64_t B,
                                                    float* __restrict__ O) {
  extern __shared__ float lds[];
  const TrainLds t = train_lds(s);
  const int lane = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * kChunk;
  chunk_forward(s, params, X, B, s0, lds, t, false, lane);
  const int nL = s.size[s.L], pL = s.pad[s.L];
  for (int e = lane; e < kChunk * nL; e += 64) {
    const int i = e / nL, j = e % nL;
    const int64_t row = s0 + i;
    if (row < B) O[row * nL + j] = lds[t.act[s.L] + i * pL + j];
  }
}

// Per-chunk gradient of loss = sum (O - T)^2 / (2 B n_out): writes the
// chunk's partial gradient (flat parameter layout) to part[blockIdx.x] and
// its share of the loss to loss_part[blockIdx.x].
__global__ __launch_bounds__(64) void k_mlp_grad(MlpShape s, const float* __restrict__ params,
                                                 const float* __restrict__ X,
                                                 const float* __restrict__ T, int64_t B,
                                                 float* __restrict__ part,
                                                 float* __restrict__ loss_part) {
  extern __shared__ float lds[];
  const TrainLds t = train_lds(s);
  const int lane = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * kChunk;
  chunk_forward(s, params, X, B, s0, lds, t, true, lane);

  // output gradient dz_L = (O - T) / (B n_L), zero on padding and on rows >= B
  const int nL = s.size[s.L], pL = s.pad[s.L];
  const float scale = 1.0f / ((float)B * (float)nL);
  float lsum = 0.0f;
  float* dz = lds + t.dz[0];
  for (int e = lane; e < kChunk * pL; e += 64) {
    const int i = e / pL, j = e % pL;
    const int64_t row = s0 + i;
    float d = 0.0f;
    if (row < B && j < nL) {
      const float diff = lds[t.act[s.L] + e] - T[row * nL + j];
      lsum += diff * diff;
      d = diff * scale;
    }
    dz[e] = d;
  }
  // wave reduction of the loss
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
  if (lane == 0) loss_part[blockIdx.x] = 0.5f * lsum * scale;
  __syncthreads();

  float* gpart = part + (int64_t)blockIdx.x * s.n_params;
  int cur = 0;
  for (int l = s.L; l >= 1; --l) {
    const int nin = s.size[l - 1], nout = s.size[l];
    const int pin = s.pad[l - 1], pout = s.pad[l];
    float* dzl = lds + t.dz[cur];
    // dW_l = dz_l^T act_{l-1}: (out x in), K = samples
    const MatRef A{dzl, 1, pout, pout, kChunk};           // (m = out, k = sample)
    const MatRef Ba{lds + t.act[l - 1], pin, 1, kChunk, pin};  // (k = sample, n = in)
    wave_gemm(A, Ba, gpart + s.w_off[l], nin, 1, nout, nin, pout, pin, kChunk, lane);
    // db_l
    for (int j = lane; j < nout; j += 64) {
      float acc = 0.0f;
      for (int i = 0; i < kChunk; ++i) acc += dzl[i * pout + j];
      gpart[s.b_off[l] + j] = acc;
    }
    if (l > 1) {
      // dA_{l-1} = dz_l W_l: (sample x in), K = out
      const float* W = params + s.w_off[l];
      float* nxt = lds + t.dz[cur ^ 1];
      const MatRef Ad{dzl, pout, 1, kChunk, pout};   // (m = sample, k = out)
      const MatRef Bw{W, nin, 1, nout, nin};          // (k = out, n = in) -> W[out][in]
      wave_gemm(Ad, Bw, nxt, pin, 1, kChunk, pin, kChunk, pin, pout, lane);
      __syncthreads();
      for (int e = lane; e < kChunk * pin; e += 64) {
        const int j = e % pin;
        nxt[e] = j < nin ? nxt[e] * act_grad(s.act, lds[t.z[l - 1] + e]) : 0.0f;
      }
      cur ^= 1;
    }
    __syncthreads();
  }
}

// Sums the chunk partials in a fixed order (deterministic) into grad, and
// the chunk losses into loss[0].
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ part, int chunks,
                                                    int64_t n_params, float* __restrict__ grad,
                                                    const float* __restrict__ loss_part,
                                                    float* __restrict__ loss) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n_params) {
    float acc = 0.0f;
    for (int c = 0; c < chunks; ++c) acc += part[(int64_t)c * n_params + p];
    grad[p] = acc;
  }
  if (p == 0 && loss) {
    float acc = 0.0f;
    for (int c = 0; c < chunks; ++c) acc += loss_part[c];
    loss[0] = acc;
  }
}

// Adam update of the FP32 master parameters.
__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ params, float* __restrict__ m,
                                                  float* __restrict__ v,
                                                  const float* __restrict__ grad, int64_t n,
                                                  float lr, float b1, float b2, float eps,
                                                  float bc1, float bc2) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float g = grad[p];
  const float mm = fmaf(b1, m[p], (1.0f - b1) * g);
  const float vv = fmaf(b2, v[p], (1.0f - b2) * g * g);
  m[p] = mm;
  v[p] = vv;
  const float mh = mm / bc1, vh = vv / bc2;
  params[p] -= lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------------------------------
// Training data: column statistics and normalization of row-major arrays
// ---------------------------------------------------------------------------

// Per-block partial statistics of the columns of A (rows x cols, row-major,
// cols <= kStatCols): block b takes rows [b rb, (b+1) rb), thread (x, y)
// column x and every kStatRows-th row from y.  Without `mean` it sums x
// and records min and max; with `mean` it sums (x - mean)^2.  FP64 sums,
// combined in a fixed order, so the statistics are deterministic.
constexpr int kStatCols = 64, kStatRows = 4;
__global__ __launch_bounds__(kStatCols * kStatRows) void k_col_partial(
    const float* __restrict__ A, int64_t rows, int cols, int64_t rb,
    const double* __restrict__ mean, double* __restrict__ part, float* __restrict__ pmin,
    float* __restrict__ pmax) {
  __shared__ double ssum[kStatRows][kStatCols];
  __shared__ float smin[kStatRows][kStatCols], smax[kStatRows][kStatCols];
  const int x = threadIdx.x, y = threadIdx.y;
  double acc = 0.0;
  float lo = __builtin_inff(), hi = -__builtin_inff();
  if (x < cols) {
    const double m = mean ? mean[x] : 0.0;
    const int64_t r0 = (int64_t)blockIdx.x * rb;
    const int64_t r1 = r0 + rb < rows ? r0 + rb : rows;
    for (int64_t r = r0 + y; r < r1; r += kStatRows) {
      const float v = A[r * cols + x];
      if (mean) {
        const double d = (double)v - m;
        acc += d * d;
      } else {
        acc += (double)v;
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
      }
    }
  }
  ssum[y][x] = acc;
  smin[y][x] = lo;
  smax[y][x] = hi;
  __syncthreads();
  if (y == 0 && x < cols) {
    for (int j = 1; j < kStatRows; ++j) {
      acc += ssum[j][x];
      lo = fminf(lo, smin[j][x]);
      hi = fmaxf(hi, smax[j][x]);
    }
    part[(int64_t)blockIdx.x * cols + x] = acc;
    if (!mean) {
      pmin[(int64_t)blockIdx.x * cols + x] = lo;
      pmax[(int64_t)blockIdx.x * cols + x] = hi;
    }
  }
}

// Sums the block partials of every column in block order: out[k] = total
// (stage 0 also min and max).
__global__ __launch_bounds__(kStatCols) void k_col_final(const double* __restrict__ part,
                                                        const float* __restrict__ pmin,
                                                        const float* __restrict__ pmax, int blocks,
                                                        int cols, double* __restrict__ out,
                                                        float* __restrict__ omin,
                                                        float* __restrict__ omax) {
  const int x = threadIdx.x;
  if (x >= cols) return;
  double acc = 0.0;
  float lo = __builtin_inff(), hi = -__builtin_inff();
  for (int b = 0; b < blocks; ++b) {
    acc += part[(int64_t)b * cols + x];
    if (omin) {
      lo = fminf(lo, pmin[(int64_t)b * cols + x]);
      hi = fmaxf(hi, pmax[(int64_t)b * cols + x]);
    }
  }
  out[x] = acc;
  if (omin) {
    omin[x] = lo;
    omax[x] = hi;
  }
}

// Y[r][k] = (A[r][k] - shift[k]) * scale[k] for k < cols, Y[r][cols] =
// extra when ldy > cols, other columns of Y untouched.
__global__ __launch_bounds__(256) void k_normalize(const float* __restrict__ A, int64_t rows,
                                                   int cols, const float* __restrict__ shift,
                                                   const float* __restrict__ scale, float extra,
                                                   float* __restrict__ Y, int ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int w = ldy > cols ? cols + 1 : cols;
  if (e >= rows * w) return;
  const int64_t r = e / w;
  const int k = (int)(e % w);
  Y[r * ldy + k] = k < cols ? (A[r * cols + k] - shift[k]) * scale[k] : extra;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_col_stats(const float* A, int64_t rows, int cols, double* part, float* pmin,
                            float* pmax, int blocks, double* sum, float* cmin, float* cmax,
                            const double* mean, double* sq, hipStream_t st) {
  const int64_t rb = (rows + blocks - 1) / blocks;
  const dim3 blk(kStatCols, kStatRows);
  hipLaunchKernelGGL(k_col_partial, dim3((unsigned)blocks), blk, 0, st, A, rows, cols, rb,
                     (const double*)nullptr, part, pmin, pmax);
  hipLaunchKernelGGL(k_col_final, dim3(1), dim3(kStatCols), 0, st, part, pmin, pmax, blocks,
                     cols, sum, cmin, cmax);
  if (mean) {
    hipLaunchKernelGGL(k_col_partial, dim3((unsigned)blocks), blk, 0, st, A, rows, cols, rb, mean,
                       part, pmin, pmax);
    hipLaunchKernelGGL(k_col_final, dim3(1), dim3(kStatCols), 0, st, part, pmin, pmax, blocks,
                       cols, sq, (float*)nullptr, (float*)nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_normalize(const float* A, int64_t rows, int cols, const float* shift,
                            const float* scale, float extra, float* Y, int ldy, hipStream_t st) {
  const int w = ldy > cols ? cols + 1 : cols;
  const int64_t n = rows * w;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_normalize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, rows,
                     cols, shift, scale, extra, Y, ldy);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpShape& s, const float* params, const float* X, int64_t B,
                              float* O, hipStream_t st) {
  if (B == 0) return hipSuccess;
  const unsigned chunks = (unsigned)((B + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_mlp_forward, dim3(chunks), dim3(64), mlp_train_lds_bytes(s), st, s, params,
                     X, B, O);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpShape& s, const float* params, const float* X, const float* T,
                           int64_t B, float* part, float* loss_part, float* grad, float* loss,
                           hipStream_t st) {
  const int chunks = (int)((B + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_mlp_grad, dim3(chunks), dim3(64), mlp_train_lds_bytes(s), st, s, params, X,
                     T, B, part, loss_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)((s.n_params + 255) / 256);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(blocks), dim3(256), 0, st, part, chunks,
                     (int64_t)s.n_params, grad, loss_part, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t n, float lr,
                           float b1, float b2, float eps, int64_t t, hipStream_t st) {
  const float bc1 = 1.0f - powf(b1, (float)t), bc2 = 1.0f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, params, m, v,
                     grad, n, lr, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

}  // namespace fib
