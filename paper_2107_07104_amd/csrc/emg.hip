// EMG step: the static bidomain solve on the structured 3D mesh (gfx950).
//
// The mesh nodes are every m-th node of an nx x ny bundle of equal fibers
// (thesis eq. discretized_fibers_2: V_3D = P V_m is an injection), and the
// elements are trilinear hexahedra with widths (hx, hy, m h).  For a
// diagonal conduction tensor D the Q1 stiffness matrix is
//   K_D = dx Kx (x) My (x) Mz + dy Mx (x) Ky (x) Mz + dz Mx (x) My (x) Kz
// with the 1D linear-element stiffness K and consistent mass M, so a row of
// K_D is a 27-point stencil whose weights are products of three 1D weights
// (each 1D factor knows whether its neighbour exists: that is the Neumann
// boundary).  The operator is applied matrix-free: no matrix is stored, the
// weights of a node are formed from its (i, j, k) in registers.
//
// A row is applied as sum_{j != t} w_tj (u_j - u_t): K_D u with the diagonal
// taken as minus the row's off-diagonal weights, which is exact for K_D
// (its rows sum to zero).  In FP32 this keeps the constant vector an exact
// null vector of the operator, as it is of K_D, so the projected Neumann
// system stays consistent and semi-definite.  Applied with the centre weight
// rounded on its own, the operator's constant mode has an eigenvalue of the
// size of the rounding and of either sign (about -3e-8 of the diagonal on a
// 3 x 7 x 121 mesh), and CG diverges once it resolves that mode.
//
// The solve (eq. discretized_fibers_3) is preconditioned conjugate gradients
// with the diagonal of K_{sigma_i + sigma_e} on the Neumann system, kept in
// the range of the operator: the stored residual r is the raw update, and
// its mean c is removed wherever it is used (z = (r - c) / diag).  Rounding
// in r -= alpha q moves the residual's sum away from zero by a random walk
// that no CG step can reduce (the constant is the operator's null vector);
// left in, it dominates r.z once the residual is small and CG diverges.
// The projected scalars come from four sums of the raw r:
//   r.z = sum r^2/d - 2 c sum r/d + c^2 sum 1/d,  r.r = sum r^2 - n c^2.
// Each iteration k is two launches:
//   k_cg_q:  the totals of the previous launch's per-block sums of r give
//            c, r.z, r.r and the convergence test; then p <- (r - c)/d +
//            beta p (the previous p in the other buffer; the stencil forms
//            its neighbours' p itself), q = A p, per-block sums of p.q;
//   k_cg_x:  alpha = r.z / p.q from the totals of those sums; x += alpha p,
//            r <- (r - c) - alpha q, per-block sums of r, r^2, r/d, r^2/d.
// Every block forms the totals itself, from FP64 per-block sums added in a
// fixed order, so all blocks agree bit for bit and every solve is
// deterministic; the kernel boundaries order the sums and scalars without
// device-wide fences.  Sums and scalars alternate between two buffers by
// the parity of k, so a launch never overwrites what its own blocks read.
// Once converged, launches return at once, so the host enqueues batches and
// checks the
// flag between them.  The grid is (blocks per layer, layers): a thread
// finds (i, j) from its index in the layer and k from the block row.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/fib.h"
#include "fib_internal.h"

namespace {

constexpr int kB = 256;  // threads per block (four waves)

struct Grid3 {
  int nx, ny, nz;
  float hx, hy, hz;
  int64_t n;
};

// Scalars of the solve, in device memory.  slot[k & 1] holds iteration
// k's projected scalars, written by block 0 of its k_cg_q.
struct Slot {
  double c;   // mean of the stored (raw) residual
  double rz;  // r.z of the projected residual
};

struct Scal {
  double mean_b;  // mean of the raw right-hand side
  double bb;      // ||b||^2 after the projection
  double sd;      // sum of 1 / diag(A)
  double tol2;    // tol^2
  double rr;      // r.r of the last residual tested
  Slot slot[2];
  int32_t it;     // iterations taken
  int32_t done;   // converged (or b = 0)
};

// Projected c, r.z, r.r from the sums of the raw residual (S1 = sum r,
// S2 = sum r^2, S1d = sum r/d, S2d = sum r^2/d).
struct Proj {
  double c, rz, rr;
};

__device__ __forceinline__ Proj project(const double* t, int64_t n, double sd) {
  const double c = t[0] / (double)n;
  return {c, fmax(t[3] - 2.0 * c * t[2] + c * c * sd, 0.0), fmax(t[1] - (double)n * c * c, 0.0)};
}

__device__ __forceinline__ bool first_thread() {
  return blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0;
}

// 1D linear-element stiffness and mass weights of node i (of n, spacing h)
// towards its neighbours i - 1, i, i + 1; a missing neighbour weighs 0.
__device__ __forceinline__ void weights_1d(int i, int n, float h, float (&K)[3], float (&M)[3]) {
  const float lo = i > 0 ? 1.0f : 0.0f, hi = i + 1 < n ? 1.0f : 0.0f;
  const float ih = 1.0f / h;
  K[0] = -lo * ih;
  K[1] = (lo + hi) * ih;
  K[2] = -hi * ih;
  M[0] = lo * h * (1.0f / 6.0f);
  M[1] = (lo + hi) * h * (1.0f / 3.0f);
  M[2] = hi * h * (1.0f / 6.0f);
}

// Row (i, j, k) of K_D applied to a field u in the difference form
// sum_{j != t} w_tj (u_j - u_t), by sum factorization over the axes:
//     dx sum_c Mz_c sum_b My_b sum_a Kx_a du
//   + dy sum_c Mz_c sum_b Ky_b sum_a Mx_a du
//   + dz sum_c Kz_c sum_b My_b sum_a Mx_a du,
// du = u(i + a - 1, j + b - 1, k + c - 1) - u(i, j, k) (the centre term is
// zero).  get(kk, l) returns u at layer kk and in-layer index l = j' nx + i'.
// A missing neighbour has 1D weight 0, and its offset is clamped to the node
// itself so that every read stays in the mesh.  diag receives the diagonal
// weight of K_D (the Jacobi preconditioner).
template <class Get>
__device__ __forceinline__ float apply_row(const Grid3& g, float dx, float dy, float dz, int i,
                                           int j, int k, Get get, float& diag) {
  float Kx[3], Mx[3], Ky[3], My[3], Kz[3], Mz[3];
  weights_1d(i, g.nx, g.hx, Kx, Mx);
  weights_1d(j, g.ny, g.hy, Ky, My);
  weights_1d(k, g.nz, g.hz, Kz, Mz);
  diag = dx * Kx[1] * My[1] * Mz[1] + dy * Mx[1] * Ky[1] * Mz[1] + dz * Mx[1] * My[1] * Kz[1];
  const uint32_t l0 = (uint32_t)(j * g.nx + i);
  const uint32_t ox[3] = {i > 0 ? ~0u : 0u, 0u, i + 1 < g.nx ? 1u : 0u};
  const uint32_t oy[3] = {j > 0 ? 0u - (uint32_t)g.nx : 0u, 0u, j + 1 < g.ny ? (uint32_t)g.nx : 0u};
  const uint32_t kz[3] = {(uint32_t)(k > 0 ? k - 1 : k), (uint32_t)k,
                          (uint32_t)(k + 1 < g.nz ? k + 1 : k)};
  const float uc = get((uint32_t)k, l0);
  float s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float y1 = 0.0f, y2 = 0.0f, y3 = 0.0f;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const uint32_t l = l0 + oy[b];
      const float d0 = get(kz[c], l + ox[0]) - uc;
      const float d1 = get(kz[c], l) - uc;
      const float d2 = get(kz[c], l + ox[2]) - uc;
      const float sk = fmaf(Kx[0], d0, fmaf(Kx[1], d1, Kx[2] * d2));
      const float sm = fmaf(Mx[0], d0, fmaf(Mx[1], d1, Mx[2] * d2));
      y1 = fmaf(My[b], sk, y1);
      y2 = fmaf(Ky[b], sm, y2);
      y3 = fmaf(My[b], sm, y3);
    }
    s1 = fmaf(Mz[c], y1, s1);
    s2 = fmaf(Mz[c], y2, s2);
    s3 = fmaf(Kz[c], y3, s3);
  }
  return fmaf(dx, s1, fmaf(dy, s2, dz * s3));
}

// Node of this thread in the (blocks per layer, layers) grid; false past
// the end of its layer.
__device__ __forceinline__ bool node_of(const Grid3& g, int& i, int& j, int& k, uint32_t& t) {
  const int tl = (int)blockIdx.x * kB + (int)threadIdx.x;  // index in the layer
  if (tl >= g.nx * g.ny) return false;
  i = tl % g.nx;
  j = tl / g.nx;
  k = (int)blockIdx.y;
  t = (uint32_t)k * (uint32_t)(g.nx * g.ny) + (uint32_t)tl;
  return true;
}

// Element idx of a vector through a 32-bit byte offset (vectors hold at
// most 2^30 elements), so that the load takes the base address from scalar
// registers and only the offset from a vector register.
__device__ __forceinline__ float at(const float* __restrict__ v, uint32_t idx) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(v) + (idx << 2));
}

// Accessor of a mesh vector for apply_row.
struct MeshVec {
  const float* __restrict__ v;
  uint32_t nxy;
  __device__ __forceinline__ float operator()(uint32_t kk, uint32_t l) const {
    return at(v, kk * nxy + l);
  }
};

// Per-block sums of NV doubles into the block's record partials[block * NV
// + v], in a fixed order (waves by shuffles, then the four waves in order).
template <int NV>
__device__ __forceinline__ void block_sums(double (&v)[NV], double* partials) {
  __shared__ double sh[NV][kB / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int blk = (int)(blockIdx.y * gridDim.x + blockIdx.x);
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double x = v[q];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x += __shfl_down(x, d);
    if (lane == 0) sh[q][wave] = x;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double x = 0.0;
    for (int w = 0; w < kB / 64; ++w) x += sh[threadIdx.x][w];
    partials[(size_t)blk * NV + threadIdx.x] = x;
  }
}

// Totals of the per-block records, the same in every block that forms them:
// thread t adds records t, t + kB, t + 2 kB, ... in that order (loaded four
// at a time, so one memory latency covers up to 4 kB blocks), then the
// waves reduce by shuffles and the four wave sums are added in order.
// Each NV has its own LDS array: one kernel must not call it twice with the
// same NV.
template <int NV>
__device__ __forceinline__ void total_sums(const double* partials, int nblocks, double (&tot)[NV]) {
  __shared__ double sh[NV][kB / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double x[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) x[q] = 0.0;
  for (int b0 = threadIdx.x; b0 < nblocks; b0 += 4 * kB) {
    double rec[4][NV];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int b = b0 + u * kB;
#pragma unroll
      for (int q = 0; q < NV; ++q) rec[u][q] = b < nblocks ? partials[(size_t)b * NV + q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int q = 0; q < NV; ++q) x[q] += rec[u][q];
    }
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x[q] += __shfl_down(x[q], d);
    if (lane == 0) sh[q][wave] = x[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double y = 0.0;
    for (int w = 0; w < kB / 64; ++w) y += sh[q][w];
    tot[q] = y;
  }
}

// b = -K_{sigma_i} P V_m from the fiber state (row 0: V_m - rest; the
// difference form sees only differences of V_m); per-block sums of b.
__global__ __launch_bounds__(kB) void k_emg_rhs(Grid3 g, const float* __restrict__ vm,
                                                int32_t n_fib, int32_t m, float sigma_i,
                                                float* __restrict__ b, double* partials) {
  int i, j, k;
  uint32_t t;
  double v[1] = {0.0};
  if (node_of(g, i, j, k, t)) {
    // 3D node (i', j', k') is fiber j' nx + i' at its node k' m
    auto get = [&](uint32_t kk, uint32_t f) {
      return at(vm, f * (uint32_t)n_fib + kk * (uint32_t)m);
    };
    float d;
    const float val = -apply_row(g, 0.0f, 0.0f, sigma_i, i, j, k, get, d);
    b[t] = val;
    v[0] = val;
  }
  block_sums<1>(v, partials);
}

__global__ __launch_bounds__(kB) void k_emg_mean(const double* partials, int nblocks, int64_t n,
                                                 Scal* s) {
  double tot[1];
  total_sums<1>(partials, nblocks, tot);
  if (threadIdx.x == 0) s->mean_b = tot[0] / (double)n;
}

// 1 / diag(A) of every node and per-block sums of it.
__global__ __launch_bounds__(kB) void k_emg_invd(Grid3 g, float dx, float dy, float dz,
                                                 float* __restrict__ invd, double* partials) {
  int i, j, k;
  uint32_t t;
  double v[1] = {0.0};
  if (node_of(g, i, j, k, t)) {
    float Kx[3], Mx[3], Ky[3], My[3], Kz[3], Mz[3];
    weights_1d(i, g.nx, g.hx, Kx, Mx);
    weights_1d(j, g.ny, g.hy, Ky, My);
    weights_1d(k, g.nz, g.hz, Kz, Mz);
    const float d = dx * Kx[1] * My[1] * Mz[1] + dy * Mx[1] * Ky[1] * Mz[1] +
                    dz * Mx[1] * My[1] * Kz[1];
    const float w = 1.0f / d;
    invd[t] = w;
    v[0] = w;
  }
  block_sums<1>(v, partials);
}

__global__ __launch_bounds__(kB) void k_emg_sd(const double* partials, int nblocks, Scal* s) {
  double tot[1];
  total_sums<1>(partials, nblocks, tot);
  if (threadIdx.x == 0) s->sd = tot[0];
}

// Sums of the raw residual rt for project(): r, r^2, r/d, r^2/d.
__device__ __forceinline__ void residual_sums(float rt, float wd, double* v) {
  const double r = rt, rw = (double)rt * wd;
  v[0] = r;
  v[1] = r * r;
  v[2] = rw;
  v[3] = rw * r;
}

// Start of CG from the last solution x: bp = b - mean(b), r = bp - A x;
// per-block sums of r, r^2, r/d, r^2/d into part_r and of bp.bp into part_b.
__global__ __launch_bounds__(kB) void k_emg_start(Grid3 g, float dx, float dy, float dz,
                                                  const float* __restrict__ b,
                                                  const float* __restrict__ x,
                                                  const float* __restrict__ invd,
                                                  float* __restrict__ r, double* part_r,
                                                  double* part_b, const Scal* s) {
  int i, j, k;
  uint32_t t;
  double v[4] = {0.0, 0.0, 0.0, 0.0}, vb[1] = {0.0};
  if (node_of(g, i, j, k, t)) {
    float d;
    const float ax = apply_row(g, dx, dy, dz, i, j, k, MeshVec{x, (uint32_t)(g.nx * g.ny)}, d);
    const float bp = b[t] - (float)s->mean_b;
    const float rt = bp - ax;
    r[t] = rt;
    residual_sums(rt, invd[t], v);
    vb[0] = (double)bp * bp;
  }
  block_sums<4>(v, part_r);
  block_sums<1>(vb, part_b);
}

__global__ __launch_bounds__(kB) void k_emg_started(const double* part_r, const double* part_b,
                                                    int nblocks, int64_t n, Scal* s) {
  double tot[4], tb[1];
  total_sums<4>(part_r, nblocks, tot);
  total_sums<1>(part_b, nblocks, tb);
  if (threadIdx.x == 0) {
    const Proj pr = project(tot, n, s->sd);
    s->bb = tb[0];
    s->rr = pr.rr;
    s->it = 0;
    s->slot[1].rz = INFINITY;  // beta = 0 in the first iteration
    s->done = (tb[0] == 0.0 || pr.rr <= s->tol2 * tb[0]) ? 1 : 0;
  }
}

// Iteration k (parity P): the test and beta from the sums of r in part_r,
// then p_new = (r - c)/d + beta p_old and q = A p_new; per-block sums of
// p.q into part_pq.
__global__ __launch_bounds__(kB) void k_cg_q(Grid3 g, float dx, float dy, float dz,
                                             const float* __restrict__ r,
                                             const float* __restrict__ invd,
                                             const float* __restrict__ p_old,
                                             float* __restrict__ p_new, float* __restrict__ q,
                                             const double* part_r, double* part_pq, int nblocks,
                                             int P, Scal* s) {
  if (s->done) return;
  double tot[4];
  total_sums<4>(part_r, nblocks, tot);
  const Proj pr = project(tot, g.n, s->sd);
  const bool done = pr.rr <= s->tol2 * s->bb;
  const double rz_prev = s->slot[P ^ 1].rz;
  if (first_thread()) {
    s->rr = pr.rr;
    s->slot[P].c = pr.c;
    s->slot[P].rz = pr.rz;
    if (done) s->done = 1;
    else s->it += 1;
  }
  if (done) return;
  const float beta = (rz_prev > 0.0 && rz_prev < INFINITY) ? (float)(pr.rz / rz_prev) : 0.0f;
  const float c = (float)pr.c;
  int i, j, k;
  uint32_t t;
  double v[1] = {0.0};
  if (node_of(g, i, j, k, t)) {
    const uint32_t nxy = (uint32_t)(g.nx * g.ny);
    auto pn = [&](uint32_t kk, uint32_t l) {
      const uint32_t n = kk * nxy + l;
      return fmaf(beta, at(p_old, n), (at(r, n) - c) * at(invd, n));
    };
    float d;
    const float qt = apply_row(g, dx, dy, dz, i, j, k, pn, d);
    const float pt = fmaf(beta, p_old[t], (r[t] - c) * invd[t]);
    p_new[t] = pt;
    q[t] = qt;
    v[0] = (double)pt * qt;
  }
  block_sums<1>(v, part_pq);
}

// Iteration k (parity P): alpha from the sums of p.q, x += alpha p,
// r <- (r - c) - alpha q; per-block sums of r, r^2, r/d, r^2/d into
// part_r (the buffer of parity P ^ 1).
__global__ __launch_bounds__(kB) void k_cg_x(Grid3 g, const float* __restrict__ p,
                                             const float* __restrict__ q,
                                             const float* __restrict__ invd,
                                             float* __restrict__ x, float* __restrict__ r,
                                             const double* part_pq, double* part_r, int nblocks,
                                             int P, const Scal* s) {
  if (s->done) return;
  double tot[1];
  total_sums<1>(part_pq, nblocks, tot);
  const float alpha = tot[0] > 0.0 ? (float)(s->slot[P].rz / tot[0]) : 0.0f;
  const float c = (float)s->slot[P].c;
  int i, j, k;
  uint32_t t;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (node_of(g, i, j, k, t)) {
    x[t] = fmaf(alpha, p[t], x[t]);
    const float rt = fmaf(-alpha, q[t], r[t] - c);
    r[t] = rt;
    residual_sums(rt, invd[t], v);
  }
  block_sums<4>(v, part_r);
}

// r.r of the last iterate when the iteration limit stopped the solve.
__global__ __launch_bounds__(kB) void k_cg_final(const double* part_r, int nblocks, int64_t n,
                                                 Scal* s) {
  if (s->done) return;
  double tot[4];
  total_sums<4>(part_r, nblocks, tot);
  if (threadIdx.x == 0) s->rr = project(tot, n, s->sd).rr;
}

// x -= mean(x): the per-block sums, the mean, the subtraction.
__global__ __launch_bounds__(kB) void k_emg_sum(Grid3 g, const float* __restrict__ x,
                                                double* partials) {
  int i, j, k;
  uint32_t t;
  double v[1] = {node_of(g, i, j, k, t) ? (double)x[t] : 0.0};
  block_sums<1>(v, partials);
}

__global__ __launch_bounds__(kB) void k_emg_shift(Grid3 g, float* __restrict__ x, const Scal* s) {
  int i, j, k;
  uint32_t t;
  if (node_of(g, i, j, k, t)) x[t] -= (float)s->mean_b;
}

int efail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return fib::set_error(code, buf);
}

#define EHIP(expr)                                                                    \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return efail(FIB_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

}  // namespace

struct fib_emg {
  fib_t* ctx = nullptr;
  fib_emg_params p{};
  Grid3 g{};
  int32_t n_fib = 0;          // nodes per fiber
  float* d_vec = nullptr;     // b, x, r, 1/diag, p0, p1, q (n each)
  double* d_part = nullptr;   // per-block sums: two of 4 x blocks (r), one of blocks (p.q)
  Scal* d_s = nullptr;
  Scal* h_s = nullptr;        // pinned copy of the scalars
  dim3 grid;                  // (blocks per layer, layers)
  int nblocks = 0;
  float* b() const { return d_vec; }
  float* x() const { return d_vec + g.n; }
  float* r() const { return d_vec + 2 * g.n; }
  float* invd() const { return d_vec + 3 * g.n; }
  float* pb(int i) const { return d_vec + (4 + i) * g.n; }
  float* q() const { return d_vec + 6 * g.n; }
  double* part_r(int par) const { return d_part + (size_t)par * 4 * nblocks; }
  double* part_pq() const { return d_part + (size_t)8 * nblocks; }
};

extern "C" {

int fib_emg_create(fib_t* ctx, const fib_emg_params* p, fib_emg_t** out) {
  if (!out) return efail(FIB_EINVAL, "null output pointer");
  *out = nullptr;
  if (!ctx || !p) return efail(FIB_EINVAL, "null argument");
  const fib::CtxView v = fib::ctx_view(ctx);
  if (p->nx < 2 || p->ny < 2 || p->stride < 1)
    return efail(FIB_EINVAL, "nx, ny must be >= 2 and the stride >= 1");
  auto pos = [](double x) { return std::isfinite(x) && x > 0.0; };
  if (!pos(p->hx) || !pos(p->hy) || !pos(p->sigma_i) || !pos(p->sigma_el) || !pos(p->sigma_et))
    return efail(FIB_EINVAL, "spacings and conductivities must be > 0");
  if ((int64_t)p->nx * p->ny != v.n_fibers)
    return efail(FIB_EINVAL, "%d x %d fibers expected, the context has %d", p->nx, p->ny,
                 v.n_fibers);
  const int32_t n = v.n_nodes[0];
  for (int32_t f = 1; f < v.n_fibers; ++f)
    if (v.n_nodes[f] != n) return efail(FIB_EINVAL, "fibers of unequal length");
  if (n < 2 || (n - 1) % p->stride != 0)
    return efail(FIB_EINVAL, "fiber length %d: (n - 1) must be a positive multiple of %d", n,
                 p->stride);
  // the kernels address the fiber state and the mesh vectors with 32-bit
  // byte offsets
  if ((int64_t)v.n_fibers * n > (int64_t(1) << 30))
    return efail(FIB_EUNSUPPORTED, "EMG bundles hold at most 2^30 fiber nodes");
  fib_emg* e = new (std::nothrow) fib_emg();
  if (!e) return efail(FIB_ENOMEM, "host allocation failed");
  e->ctx = ctx;
  e->p = *p;
  e->n_fib = n;
  e->g.nx = p->nx;
  e->g.ny = p->ny;
  e->g.nz = (n - 1) / p->stride + 1;
  e->g.hx = (float)p->hx;
  e->g.hy = (float)p->hy;
  e->g.hz = (float)(p->stride * v.h);
  e->g.n = (int64_t)e->g.nx * e->g.ny * e->g.nz;
  e->grid = dim3((unsigned)((e->g.nx * e->g.ny + kB - 1) / kB), (unsigned)e->g.nz);
  e->nblocks = (int)(e->grid.x * e->grid.y);
  const size_t nv = (size_t)e->g.n * 7;
  if (hipMalloc(&e->d_vec, sizeof(float) * nv) != hipSuccess ||
      hipMalloc(&e->d_part, sizeof(double) * 9 * e->nblocks) != hipSuccess ||
      hipMalloc(&e->d_s, sizeof(Scal)) != hipSuccess ||
      hipHostMalloc(&e->h_s, sizeof(Scal)) != hipSuccess) {
    fib_emg_destroy(e);
    return efail(FIB_ENOMEM, "device allocation failed");
  }
  // zeros (x = 0 is the first solve's start), then 1/diag(A) and its sum,
  // all on the context's stream
  hipStream_t st = v.stream;
  bool ok = hipMemsetAsync(e->d_vec, 0, sizeof(float) * nv, st) == hipSuccess &&
            hipMemsetAsync(e->d_s, 0, sizeof(Scal), st) == hipSuccess;
  if (ok) {
    hipLaunchKernelGGL(k_emg_invd, e->grid, dim3(kB), 0, st, e->g, (float)p->sigma_et,
                       (float)p->sigma_et, (float)(p->sigma_el + p->sigma_i), e->invd(),
                       e->d_part);
    hipLaunchKernelGGL(k_emg_sd, dim3(1), dim3(kB), 0, st, e->d_part, e->nblocks, e->d_s);
    ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(st) == hipSuccess;
  }
  if (!ok) {
    fib_emg_destroy(e);
    return efail(FIB_EHIP, "device initialisation failed");
  }
  *out = e;
  return FIB_OK;
}

void fib_emg_destroy(fib_emg_t* e) {
  if (!e) return;
  (void)hipFree(e->d_vec);
  (void)hipFree(e->d_part);
  (void)hipFree(e->d_s);
  if (e->h_s) (void)hipHostFree(e->h_s);
  delete e;
}

int fib_emg_dims(const fib_emg_t* e, int32_t* nx, int32_t* ny, int32_t* nz) {
  if (!e) return efail(FIB_EINVAL, "null EMG handle");
  if (nx) *nx = e->g.nx;
  if (ny) *ny = e->g.ny;
  if (nz) *nz = e->g.nz;
  return FIB_OK;
}

int fib_emg_solve(fib_emg_t* e, double tol, int32_t max_iter, int32_t* iters, double* rel_res) {
  if (!e) return efail(FIB_EINVAL, "null EMG handle");
  if (!(std::isfinite(tol) && tol > 0.0) || max_iter < 0)
    return efail(FIB_EINVAL, "tol must be > 0 and max_iter >= 0");
  const fib::CtxView v = fib::ctx_view(e->ctx);
  if (!v.state_ready) return efail(FIB_ESTATE, "state not initialized");
  hipStream_t st = v.stream;
  const Grid3 g = e->g;
  const float dx = (float)e->p.sigma_et, dy = (float)e->p.sigma_et,
              dz = (float)(e->p.sigma_el + e->p.sigma_i);
  const dim3 grid = e->grid, block(kB), one(1);
  const int nb = e->nblocks;
  // the tolerance; the host bounds the iterations
  e->h_s->tol2 = tol * tol;
  EHIP(hipMemcpyAsync(&e->d_s->tol2, &e->h_s->tol2, sizeof(double), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_emg_rhs, grid, block, 0, st, g, v.d_state, e->n_fib, e->p.stride,
                     (float)e->p.sigma_i, e->b(), e->d_part);
  hipLaunchKernelGGL(k_emg_mean, one, block, 0, st, e->d_part, nb, g.n, e->d_s);
  hipLaunchKernelGGL(k_emg_start, grid, block, 0, st, g, dx, dy, dz, e->b(), e->x(),
                     e->invd(), e->r(), e->part_r(0), e->part_pq(), e->d_s);
  hipLaunchKernelGGL(k_emg_started, one, block, 0, st, e->part_r(0), e->part_pq(), nb, g.n,
                     e->d_s);
  EHIP(hipGetLastError());
  // Iterations in batches between host checks.  The first batch is 8; then
  // the residual's mean decay rate over the last batch predicts how many
  // iterations remain, and the next batch is that (+ 25 %, at most 64), so
  // a solve wastes few no-op launches past convergence and few round trips.
  int32_t launched = 0;
  int batch = 8;
  double rr_last = -1.0;
  int32_t it_last = 0;
  for (;;) {
    EHIP(hipMemcpyAsync(e->h_s, e->d_s, sizeof(Scal), hipMemcpyDeviceToHost, st));
    EHIP(hipStreamSynchronize(st));
    if (e->h_s->done || launched >= max_iter) break;
    const double rr = e->h_s->rr, goal = e->h_s->tol2 * e->h_s->bb;
    if (rr_last > 0.0 && rr > 0.0 && rr < rr_last && e->h_s->it > it_last) {
      const double per_it = std::log(rr / rr_last) / (double)(e->h_s->it - it_last);
      const double need = std::log(goal / rr) / per_it;  // > 0: rr > goal here
      batch = (int)std::min(64.0, std::max(2.0, std::ceil(1.25 * need) + 1.0));
    } else if (rr_last > 0.0) {
      batch = std::min(2 * batch, 64);
    }
    rr_last = rr;
    it_last = e->h_s->it;
    const int n_it = std::min(batch, max_iter - launched);
    for (int b = 0; b < n_it; ++b) {
      const int P = (launched + b) & 1;
      hipLaunchKernelGGL(k_cg_q, grid, block, 0, st, g, dx, dy, dz, e->r(), e->invd(),
                         e->pb(P), e->pb(P ^ 1), e->q(), e->part_r(P), e->part_pq(), nb, P,
                         e->d_s);
      hipLaunchKernelGGL(k_cg_x, grid, block, 0, st, g, e->pb(P ^ 1), e->q(), e->invd(),
                         e->x(), e->r(), e->part_pq(), e->part_r(P ^ 1), nb, P, e->d_s);
    }
    EHIP(hipGetLastError());
    launched += n_it;
  }
  if (!e->h_s->done && launched > 0) {
    // stopped by the limit: the residual of the last iterate
    hipLaunchKernelGGL(k_cg_final, one, block, 0, st, e->part_r(launched & 1), nb, g.n, e->d_s);
    EHIP(hipGetLastError());
    EHIP(hipMemcpyAsync(e->h_s, e->d_s, sizeof(Scal), hipMemcpyDeviceToHost, st));
    EHIP(hipStreamSynchronize(st));
  }
  const int32_t done_it = e->h_s->it;
  if (e->h_s->bb == 0.0) {
    // b = 0: phi_e is a constant, zero after the projection
    EHIP(hipMemsetAsync(e->x(), 0, sizeof(float) * g.n, st));
  } else {
    hipLaunchKernelGGL(k_emg_sum, grid, block, 0, st, g, e->x(), e->d_part);
    hipLaunchKernelGGL(k_emg_mean, one, block, 0, st, e->d_part, nb, g.n, e->d_s);
    hipLaunchKernelGGL(k_emg_shift, grid, block, 0, st, g, e->x(), e->d_s);
    EHIP(hipGetLastError());
  }
  EHIP(hipStreamSynchronize(st));
  if (iters) *iters = done_it;
  if (rel_res) *rel_res = e->h_s->bb > 0.0 ? std::sqrt(e->h_s->rr / e->h_s->bb) : 0.0;
  return FIB_OK;
}

int fib_emg_get_phi(fib_emg_t* e, double* phi, int64_t n) {
  if (!e) return efail(FIB_EINVAL, "null EMG handle");
  if (n != e->g.n || !phi) return efail(FIB_EINVAL, "expected %lld values", (long long)e->g.n);
  std::vector<float> h(n);
  EHIP(hipStreamSynchronize(fib::ctx_view(e->ctx).stream));
  EHIP(hipMemcpy(h.data(), e->x(), sizeof(float) * n, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n; ++i) phi[i] = h[i];
  return FIB_OK;
}

int fib_emg_get_rhs(fib_emg_t* e, double* rhs, int64_t n) {
  if (!e) return efail(FIB_EINVAL, "null EMG handle");
  if (n != e->g.n || !rhs) return efail(FIB_EINVAL, "expected %lld values", (long long)e->g.n);
  std::vector<float> h(n);
  EHIP(hipStreamSynchronize(fib::ctx_view(e->ctx).stream));
  EHIP(hipMemcpy(h.data(), e->b(), sizeof(float) * n, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n; ++i) rhs[i] = h[i];
  return FIB_OK;
}

}  // extern "C"
