// Host runtime of libfib.so: the C ABI declared in include/fib.h.
//
// Responsibilities: argument checking, device buffers, the fiber-to-bin
// plan of the fused / diffusion kernels, the stimulus tables, kernel
// launches on the caller's stream, and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <queue>
#include <string>
#include <utility>
#include <deque>
#include <vector>

#include "../../include/fib.h"
#include "fib_internal.h"
#include "mlp_internal.h"
#include "st57_model.h"
#include "surrogate_internal.h"

using fib::KArgs;

namespace {
thread_local std::string g_err;
}  // namespace

namespace fib {
// Records an error message for fib_last_error() and returns `code`.
int set_error(int code, const char* msg) {
  g_err = msg;
  return code;
}
}  // namespace fib

namespace {

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(FIB_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int n_states_of(int model) {
  if (model == FIB_MODEL_HH || model == FIB_MODEL_HH_APX_EXP) return 4;
  if (model == FIB_MODEL_ST57 || model == FIB_MODEL_ST57_APX) return fib::st57::S;
  return -1;
}

// ---------------------------------------------------------------------------
// Hodgkin-Huxley resting state on the host (FP64)
// ---------------------------------------------------------------------------

// Equilibrium gate values at voltage V and the ionic current they carry
// (apx: exp replaced by exp*(x) = (1 + x/1024)^1024 = exp(1024 log1p(x/1024))).
double hh_steady_current(double V, double gates[3], bool apx = false) {
  const double v = V + 75.0;
  auto ex = [apx](double x) { return apx ? std::exp(1024.0 * std::log1p(x / 1024.0)) : std::exp(x); };
  auto em1 = [apx](double x) { return apx ? std::expm1(1024.0 * std::log1p(x / 1024.0)) : std::expm1(x); };
  auto lin = [&](double x) { return std::fabs(x) < 1e-6 ? 1.0 - 0.5 * x : x / em1(x); };
  const double am = lin((25.0 - v) / 10.0);
  const double bm = 4.0 * ex(-v / 18.0);
  const double ah = 0.07 * ex(-v / 20.0);
  const double bh = 1.0 / (ex((30.0 - v) / 10.0) + 1.0);
  const double an = 0.1 * lin((10.0 - v) / 10.0);
  const double bn = 0.125 * ex(-v / 80.0);
  const double m = am / (am + bm), h = ah / (ah + bh), n = an / (an + bn);
  gates[0] = m;
  gates[1] = h;
  gates[2] = n;
  return 120.0 * m * m * m * h * (V - 40.0) + 36.0 * n * n * n * n * (V + 87.0) +
         0.3 * (V + 64.387);
}

// Newton's method on the steady-state current with a central-difference
// derivative, started at the nominal resting potential of -75 mV.
int hh_rest(double* y, bool apx = false) {
  double g[3];
  double V = -75.0;
  for (int it = 0; it < 50; ++it) {
    const double f = hh_steady_current(V, g, apx);
    const double e = 1e-6;
    const double df =
        (hh_steady_current(V + e, g, apx) - hh_steady_current(V - e, g, apx)) / (2 * e);
    if (!(df > 0.0)) return fail(FIB_EINVAL, "resting-state search: non-positive slope");
    const double dV = f / df;
    V -= dV;
    if (std::fabs(dV) < 1e-13) break;
  }
  hh_steady_current(V, g, apx);
  y[0] = V;
  y[1] = g[0];
  y[2] = g[1];
  y[3] = g[2];
  return FIB_OK;
}

// ---------------------------------------------------------------------------
// ST57 resting state on the host (FP64): Newton's method on G(y) = 0 where
// one equation of each conserving block is replaced by its conserved sum
// (four probability chains sum to 1, total Ca 2200 uM, total Mg 1500 uM),
// finite-difference Jacobian, LU with partial pivoting, step halving.
// ---------------------------------------------------------------------------

constexpr int kS57 = fib::st57::S;

void st57_residual(bool apx, const std::vector<double>& y, std::vector<double>& F) {
  double u[kS57], d[kS57], zero[kS57];
  for (int k = 0; k < kS57; ++k) {
    u[k] = y[k];
    zero[k] = 0.0;
  }
  if (apx)
    fib::st57::rhs<double, true>(u, zero, 0.0, 1.0, d);
  else
    fib::st57::rhs<double, false>(u, zero, 0.0, 1.0, d);
  for (int k = 0; k < kS57; ++k) F[k] = d[k];
  auto sum = [&](int a, int b) {
    double s = 0.0;
    for (int i = a; i <= b; ++i) s += y[i];
    return s;
  };
  F[8] = sum(8, 17) - 1.0;
  F[35] = sum(35, 38) - 1.0;
  F[39] = sum(39, 46) - 1.0;
  F[47] = sum(47, 54) - 1.0;
  F[21] = y[18] + y[21] + y[22] + y[24] + 0.1 * (y[19] + y[27]) + 0.01 * (y[20] + y[28]) - 2200.0;
  F[23] = y[26] + y[23] + y[25] - 1500.0;
}

int lu_solve(std::vector<double>& A, std::vector<double>& b, int n) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[(size_t)i * n + k]) > std::fabs(A[(size_t)p * n + k])) p = i;
    if (A[(size_t)p * n + k] == 0.0) return -1;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
      std::swap(b[k], b[p]);
    }
    for (int i = k + 1; i < n; ++i) {
      const double f = A[(size_t)i * n + k] / A[(size_t)k * n + k];
      A[(size_t)i * n + k] = 0.0;
      for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < n; ++j) s -= A[(size_t)i * n + j] * b[j];
    b[i] = s / A[(size_t)i * n + i];
  }
  return 0;
}

int st57_rest(double* out, bool apx = false) {
  std::vector<double> y(kS57, 0.0), F(kS57), Fp(kS57), yp(kS57), J((size_t)kS57 * kS57),
      dx(kS57);
  // start: membranes at -75 mV with Hodgkin-Huxley resting gates, every
  // probability chain uniform, resting free Ca 0.05 uM, SR Ca 1000 uM with
  // buffers half loaded, ions at their targets
  const double hh0[4] = {-75.0, 0.05, 0.6, 0.32};
  for (int k = 0; k < 4; ++k) y[k] = y[4 + k] = hh0[k];
  for (int i = 8; i <= 17; ++i) y[i] = 0.1;
  y[18] = 0.05;
  y[19] = y[20] = 1000.0;
  y[21] = 5.0;
  y[22] = 500.0;
  y[23] = 500.0;
  y[24] = 2.0;
  y[25] = 500.0;
  y[26] = 500.0;
  y[27] = y[28] = 12000.0;
  y[29] = 10.0;
  y[30] = 140.0;
  y[31] = 5.0;
  y[32] = 140.0;
  y[33] = 5.0;
  y[34] = 128.0;
  for (int i = 35; i <= 38; ++i) y[i] = 0.25;
  for (int i = 39; i <= 54; ++i) y[i] = 0.125;
  y[55] = 1.1;
  for (int it = 0; it < 300; ++it) {
    st57_residual(apx, y, F);
    double nrm = 0.0;
    for (double f : F) nrm = std::max(nrm, std::fabs(f));
    if (nrm < 1e-11) {
      for (int k = 0; k < kS57; ++k) out[k] = y[k];
      return FIB_OK;
    }
    for (int j = 0; j < kS57; ++j) {
      yp = y;
      const double e = 1e-7 * std::max(1.0, std::fabs(y[j]));
      yp[j] += e;
      st57_residual(apx, yp, Fp);
      for (int i = 0; i < kS57; ++i) J[(size_t)i * kS57 + j] = (Fp[i] - F[i]) / e;
    }
    for (int i = 0; i < kS57; ++i) dx[i] = -F[i];
    if (lu_solve(J, dx, kS57)) return fail(FIB_EINVAL, "ST57 resting state: singular Jacobian");
    double lam = 1.0;
    for (int k = 0; k < 50; ++k, lam *= 0.5) {
      bool ok = true;
      for (int i = 0; i < kS57; ++i) {
        yp[i] = y[i] + lam * dx[i];
        if (i >= 8 && i <= 54 && yp[i] < 0.0) ok = false;
      }
      if (!ok) continue;
      st57_residual(apx, yp, Fp);
      double np = 0.0;
      for (double f : Fp) np = std::max(np, std::fabs(f));
      if (np < nrm) break;
    }
    y = yp;
  }
  return fail(FIB_EINVAL, "ST57 resting state: Newton did not converge");
}

int64_t ceil_steps(double span, double dt) {
  const double n = std::ceil(span / dt - 1e-9);
  return n < 1.0 ? 1 : (int64_t)n;
}


}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------

struct fib_ctx {
  fib_params p{};
  int S = 0;
  int32_t n_fibers = 0;
  std::vector<int32_t> n_nodes;
  std::vector<int64_t> offsets;
  int64_t n_total = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  int cu_count = 0;
  size_t max_lds = 0;
  double rest[fib::MAX_STATES] = {};

  // plan
  int groups = 0, threads = 0, K = 0, cap = 0, levels = 0;
  std::vector<int32_t> slot_gidx;      // groups * cap
  std::vector<uint32_t> slot_base;     // coupling and real-node bits
  std::vector<std::vector<int32_t>> bin_fibers;
  // fiber entries of the bins (KArgs::bin_ent and following)
  std::vector<int32_t> bin_ent, ent_s0, ent_gofs, ent_fiber;
  int32_t max_ents = 1;
  // PCR levels of fib_step_diffusion's last span (for the plan version)
  uint64_t lv_cache_version = ~0ull;
  double lv_cache_r = -1.0;
  int lv_cache_levels = 0;

  // device buffers
  float* d_state = nullptr;
  float* d_tact = nullptr;
  float* d_vprev = nullptr;
  int* d_flag = nullptr;
  int32_t* d_slot_gidx = nullptr;
  uint32_t* d_slot_info = nullptr;
  int32_t* d_bin_ent = nullptr;  // bin_ent, then ent_s0, ent_gofs, ent_fiber
  size_t ent_alloc = 0;          // int32 values in d_bin_ent
  int32_t* d_node_stim = nullptr;
  fib::StimDev* d_stim = nullptr;
  int32_t n_stim = 0;
  std::vector<int32_t> node_stim;      // host copy: stimulus entry + 1 per node (0: none)
  bool state_ready = false;
  bool tune_pending = false;  // fib_params.tune: autotune before the first run

  // surrogate
  bool sur_on = false;
  fib::SurrogateNet sur_net{};
  fib::SurrogateScales sur_sc{};
  __bf16* d_sur_frags = nullptr;
  float* d_sur_bias = nullptr;
  float* d_sur_tab = nullptr;
  int* d_sur_list = nullptr;
  int* d_sur_count = nullptr;  // two counters, alternated between surrogate steps
  int sur_slot = 0;             // counter of the next surrogate step
  int sur_last_slot = -1;       // counter of the last one (-1: none yet)
  int sur_grid = 0;
  int sur_pred = FIB_PRED_NETWORK;            // predictor of the attached step
  unsigned long long* d_sur_total = nullptr;  // rejections since the step was attached
  int64_t sur_steps = 0;                      // surrogate steps since then

  // adaptive computation (split schedule)
  double adapt_tol = 0.0;              // > 0: on
  std::vector<int32_t> first_on;       // per fiber: first step with a stimulus entry on
  int32_t* d_node_fiber = nullptr;     // [n_total]
  int32_t* d_first_on = nullptr;       // [n_fibers]
  uint8_t* d_pt = nullptr;             // [2][n_total] point flags by step parity
  uint8_t* d_fiber_any = nullptr;      // [2][n_fibers] by step parity
  unsigned long long* d_adapt_count = nullptr;  // [kAdaptCounters]
  int32_t* d_adapt_list = nullptr;     // ST57: [n_total] nodes solved in the step
  int32_t* d_adapt_lcount = nullptr;   // ST57: [2] list lengths by step parity
  int adapt_par = 0;                   // parity of the buffer with the latest flags
  // tables of the adaptive fused kernel, valid for plan / stimulus versions
  uint8_t* d_slot_fiber = nullptr;     // [groups * cap] bin-local fiber of each slot
  int32_t* d_bin_first_on = nullptr;   // [groups * kBinFibers]
  size_t adapt_slots = 0, adapt_bins = 0;  // allocated sizes
  uint64_t plan_version = 0, stim_version = 0;
  uint64_t adapt_tables_plan = ~0ull, adapt_tables_stim = ~0ull;
  bool adapt_fused_ok = false;

  // kernel timing (fib_set_kernel_timing): HIP event pairs around launches,
  // harvested in order once they have completed
  struct KtRec {
    int cls;
    hipEvent_t a, b;
    bool own_a, own_b;  // the events go back to the pool with this record
  };
  bool kt_on = false;
  std::deque<KtRec> kt_pending;
  // graph replay of the split schedule (fib_set_graphs)
  bool graphs = true;
  hipStream_t cap_stream = nullptr;      // non-blocking stream the blocks are captured on
  int32_t* d_step_base = nullptr;        // device step base of the replays
  hipGraph_t graph = nullptr;            // the last captured block and its executable,
  hipGraphExec_t graph_exec = nullptr;   // kept until its replays have completed
  hipEvent_t graph_done = nullptr;       // recorded after the last replay of graph_exec
  int64_t graph_replays = 0;
  std::vector<hipEvent_t> kt_pool;
  double kt_ms[FIB_KT_COUNT] = {};
  int64_t kt_n[FIB_KT_COUNT] = {};
};

namespace fib {
CtxView ctx_view(const fib_ctx* c) {
  CtxView v{};
  v.n_fibers = c->n_fibers;
  v.n_nodes = c->n_nodes.data();
  v.n_total = c->n_total;
  v.d_state = c->d_state;
  v.h = c->p.h;
  v.stream = c->stream;
  v.state_ready = c->state_ready;
  v.model = c->p.model;
  return v;
}
}  // namespace fib

namespace {

// Packs fibers into `groups` bins: longest-processing-time-first (fibers in
// order of decreasing length, each into the currently lightest bin), then
// pairwise moves and swaps out of the heaviest bin while they lower it.
// Every workgroup runs the same number of slots, so the heaviest bin sets
// the slots per thread of the whole launch.
void pack_bins(fib_ctx* c, int groups) {
  std::vector<int32_t> order(c->n_fibers);
  for (int32_t f = 0; f < c->n_fibers; ++f) order[f] = f;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return c->n_nodes[a] > c->n_nodes[b]; });
  using Item = std::pair<int64_t, int>;  // (load, bin)
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  for (int b = 0; b < groups; ++b) heap.push({0, b});
  c->bin_fibers.assign(groups, {});
  for (int32_t f : order) {
    Item it = heap.top();
    heap.pop();
    c->bin_fibers[it.second].push_back(f);
    heap.push({it.first + c->n_nodes[f], it.second});
  }
  // refinement
  std::vector<int64_t> load(groups, 0);
  for (int b = 0; b < groups; ++b)
    for (int32_t f : c->bin_fibers[b]) load[b] += c->n_nodes[f];
  for (int iter = 0; iter < 20000; ++iter) {
    const int hb = (int)(std::max_element(load.begin(), load.end()) - load.begin());
    const int64_t top = load[hb];
    int64_t best = top;
    int bb = -1, bi = -1, bj = -1;  // bin, index in hb, index in bb (-1: move)
    for (int b = 0; b < groups; ++b) {
      if (b == hb) continue;
      for (int i = 0; i < (int)c->bin_fibers[hb].size(); ++i) {
        const int64_t a = c->n_nodes[c->bin_fibers[hb][i]];
        // move a to b
        const int64_t mv = std::max(top - a, load[b] + a);
        if (mv < best) { best = mv; bb = b; bi = i; bj = -1; }
        for (int j = 0; j < (int)c->bin_fibers[b].size(); ++j) {
          const int64_t d = a - c->n_nodes[c->bin_fibers[b][j]];
          if (d <= 0) continue;
          const int64_t sw = std::max(top - d, load[b] + d);
          if (sw < best) { best = sw; bb = b; bi = i; bj = j; }
        }
      }
    }
    if (bb < 0) break;
    const int32_t fa = c->bin_fibers[hb][bi];
    if (bj < 0) {
      c->bin_fibers[hb].erase(c->bin_fibers[hb].begin() + bi);
      c->bin_fibers[bb].push_back(fa);
      load[hb] -= c->n_nodes[fa];
      load[bb] += c->n_nodes[fa];
    } else {
      const int32_t fb = c->bin_fibers[bb][bj];
      c->bin_fibers[hb][bi] = fb;
      c->bin_fibers[bb][bj] = fa;
      const int64_t d = c->n_nodes[fa] - c->n_nodes[fb];
      load[hb] -= d;
      load[bb] += d;
    }
  }
}

// Reduced-system coefficients (Ra, Rd, Rc) of every thread of one bin in
// FP64, the same quantities the kernels derive in FP32; used to pick the
// number of PCR levels after which every remaining coupling is below
// 2^-40 of its diagonal.
int pcr_levels_needed(const fib_ctx* c, int bin, double r, bool full) {
  const int T = c->threads, K = c->K;
  const int full_levels = (int)std::ceil(std::log2((double)T) - 1e-12);
  if (full) return full_levels;
  std::vector<double> Ra(T), Rd(T), Rc(T), v0(T), w0(T), vL(T), wL(T), ae(T), ce(T), de(T);
  constexpr int KM = 16;  // nodes per thread of any built shape (at most 14)
  if (K > KM) return full_levels;
  for (int t = 0; t < T; ++t) {
    double a[KM], cc[KM], d[KM];
    for (int q = 0; q < K; ++q) {
      const uint32_t info = c->slot_base[(size_t)bin * c->cap + (size_t)t * K + q];
      const bool L = info & fib::SLOT_L, R = info & fib::SLOT_R;
      const double wl = L ? (R ? 0.5 * r : r) : 0.0, wr = R ? (L ? 0.5 * r : r) : 0.0;
      a[q] = -wl;
      cc[q] = -wr;
      d[q] = 1.0 + wl + wr;
    }
    // interior responses to z_{t-1} (v) and z_t (w) by dense elimination
    const int m = K - 1;
    double inv[KM], cp[KM], vp[KM], v[KM], w[KM];
    for (int q = 0; q < m; ++q) {
      const double den = q == 0 ? d[0] : d[q] - a[q] * cp[q - 1];
      inv[q] = 1.0 / den;
      cp[q] = cc[q] * inv[q];
      vp[q] = q == 0 ? -a[0] * inv[0] : -a[q] * vp[q - 1] * inv[q];
    }
    v[m - 1] = vp[m - 1];
    w[m - 1] = -cp[m - 1];
    for (int q = m - 2; q >= 0; --q) {
      v[q] = vp[q] - cp[q] * v[q + 1];
      w[q] = -cp[q] * w[q + 1];
    }
    v0[t] = v[0];
    w0[t] = w[0];
    vL[t] = v[m - 1];
    wL[t] = w[m - 1];
    ae[t] = a[K - 1];
    ce[t] = cc[K - 1];
    de[t] = d[K - 1];
  }
  for (int t = 0; t < T; ++t) {
    const double vn = t + 1 < T ? v0[t + 1] : 0.0, wn = t + 1 < T ? w0[t + 1] : 0.0;
    Ra[t] = ae[t] * vL[t];
    Rd[t] = de[t] + ae[t] * wL[t] + ce[t] * vn;
    Rc[t] = ce[t] * wn;
  }
  const double tol = std::ldexp(1.0, -40);
  auto coupling = [&]() {
    double mu = 0.0;
    for (int t = 0; t < T; ++t) mu = std::max(mu, (std::fabs(Ra[t]) + std::fabs(Rc[t])) / std::fabs(Rd[t]));
    return mu;
  };
  int l = 0;
  while (l < full_levels && coupling() > tol) {
    const int s = 1 << l;
    std::vector<double> na(T), nd(T), nc(T);
    for (int t = 0; t < T; ++t) {
      const bool hl = t - s >= 0, hr = t + s < T;
      const double ra_l = hl ? Ra[t - s] : 0.0, rd_l = hl ? Rd[t - s] : 1.0, rc_l = hl ? Rc[t - s] : 0.0;
      const double ra_r = hr ? Ra[t + s] : 0.0, rd_r = hr ? Rd[t + s] : 1.0, rc_r = hr ? Rc[t + s] : 0.0;
      const double al = -Ra[t] / rd_l, ga = -Rc[t] / rd_r;
      nd[t] = Rd[t] + al * rc_l + ga * ra_r;
      na[t] = al * ra_l;
      nc[t] = ga * rc_r;
    }
    Ra.swap(na);
    Rd.swap(nd);
    Rc.swap(nc);
    ++l;
  }
  return l;
}

// The most PCR levels any bin needs for row weight r.  Bins with the same
// sequence of fiber lengths have the same matrix, so each distinct sequence
// is evaluated once.
int max_pcr_levels(const fib_ctx* c, double r) {
  std::map<std::vector<int32_t>, int> seen;
  int lv = 0;
  for (int b = 0; b < c->groups; ++b) {
    std::vector<int32_t> key;
    key.reserve(c->bin_fibers[b].size());
    for (int32_t f : c->bin_fibers[b]) key.push_back(c->n_nodes[f]);
    auto it = seen.find(key);
    if (it == seen.end())
      it = seen.emplace(std::move(key), pcr_levels_needed(c, b, r, c->p.pcr_full != 0)).first;
    lv = std::max(lv, it->second);
  }
  return lv;
}

double cn_r(const fib_ctx* c, double dt_cn) {
  return c->p.sigma / (c->p.Am * c->p.Cm) * dt_cn / (c->p.h * c->p.h);
}

// theta of the diffusion substeps' theta-scheme
double theta_of(const fib_params& p) { return p.time_1d == FIB_1D_IMPLICIT_EULER ? 1.0 : 0.5; }

// Diffusion coefficients of a launch with substep dt_cn: r_mat = 2 theta r
// (r = c dt_cn / h^2) gives the row weights of the matrix I - theta dt L,
// and 1 / theta times them the right-hand side dt L V.
void set_diffusion(const fib_ctx* c, double dt_cn, KArgs& a) {
  const double r = cn_r(c, dt_cn);
  a.r_mat = (float)(2.0 * theta_of(c->p) * r);
  a.rhs = (float)(1.0 / theta_of(c->p));
}

// Fills the slot tables and the PCR level count of the current shape
// (groups, threads, K) and bins.
void build_tables(fib_ctx* c) {
  ++c->plan_version;
  c->cap = c->threads * c->K;
  const size_t nslots = (size_t)c->groups * c->cap;
  c->slot_gidx.assign(nslots, -1);
  c->slot_base.assign(nslots, 0u);
  for (int b = 0; b < c->groups; ++b) {
    size_t pos = (size_t)b * c->cap;
    for (int32_t f : c->bin_fibers[b]) {
      const int32_t n = c->n_nodes[f];
      for (int32_t j = 0; j < n; ++j) {
        uint32_t info = fib::SLOT_REAL;
        if (j > 0) info |= fib::SLOT_L;
        if (j + 1 < n) info |= fib::SLOT_R;
        c->slot_gidx[pos] = (int32_t)(c->offsets[f] + j);
        c->slot_base[pos] = info;
        ++pos;
      }
    }
  }
  c->bin_ent.assign(1, 0);
  c->ent_s0.clear();
  c->ent_gofs.clear();
  c->ent_fiber.clear();
  c->max_ents = 1;
  for (int b = 0; b < c->groups; ++b) {
    int32_t s0 = 0;
    for (int32_t f : c->bin_fibers[b]) {
      c->ent_s0.push_back(s0);
      c->ent_gofs.push_back((int32_t)c->offsets[f]);
      c->ent_fiber.push_back(f);
      s0 += c->n_nodes[f];
    }
    c->ent_s0.push_back(s0);  // end entry: the bin's load
    c->ent_gofs.push_back(0);
    c->ent_fiber.push_back(0);
    c->bin_ent.push_back((int32_t)c->ent_s0.size());
    c->max_ents = std::max<int32_t>(c->max_ents, (int32_t)c->bin_fibers[b].size() + 1);
  }
  // PCR levels for the matrix of the split step's diffusion substep
  const int64_t n_cn = ceil_steps(c->p.dt_split, c->p.dt_1D);
  const double r = 2.0 * theta_of(c->p) * cn_r(c, c->p.dt_split / (double)n_cn);
  c->levels = max_pcr_levels(c, r);
}

int64_t max_bin_load(const fib_ctx* c) {
  int64_t load = 0;
  for (auto& b : c->bin_fibers) {
    int64_t s = 0;
    for (int32_t f : b) s += c->n_nodes[f];
    load = std::max(load, s);
  }
  return std::max<int64_t>(load, 1);
}

// Chooses bins, threads per bin and nodes per thread, and fills the slot
// tables.  Automatic shapes use K <= 8 nodes per thread; fib_autotune
// measures the others.
//  * Contexts that may run the fused schedule (Hodgkin-Huxley, schedule
//    auto or fused) get one bin per compute unit if the fibers fit: the
//    fused kernel keeps every state of its bin in registers for the whole
//    run, and a power-of-two workgroup.
//  * Split-schedule contexts (ST57 models, or schedule split) only run the
//    diffusion with bins: many small bins (one fiber each if fibers have
//    1024 nodes or more, else about 2048 nodes) of at least 4 nodes per
//    thread keep several workgroups resident per compute unit, so one
//    bin's loads overlap another's solve.
int make_plan(fib_ctx* c) {
  const int64_t max_len =
      c->n_fibers ? *std::max_element(c->n_nodes.begin(), c->n_nodes.end()) : 0;
  int64_t max_hold = 0;  // the most nodes one workgroup of any built shape holds
  for (int K = 2; K <= 14; ++K)
    max_hold = std::max<int64_t>(max_hold, (int64_t)K * fib::plan_max_threads(K));
  if (max_len > max_hold)
    return fail(FIB_EUNSUPPORTED, "fiber of %lld nodes exceeds the %lld nodes one workgroup holds",
                (long long)max_len, (long long)max_hold);
  const bool hh_like = c->p.model == FIB_MODEL_HH || c->p.model == FIB_MODEL_HH_APX_EXP;
  const bool split_plan = !hh_like || c->p.schedule == FIB_SCHED_SPLIT;
  int groups = c->p.groups > 0 ? c->p.groups : c->cu_count;
  if (split_plan && c->p.groups <= 0)
    groups = (int)std::min<int64_t>(
        INT32_MAX, max_len >= 1024 ? c->n_fibers : (c->n_total + 2047) / 2048);
  groups = (int)std::min<int64_t>(groups, std::max<int32_t>(c->n_fibers, 1));
  groups = std::max(groups, 1);
  for (;;) {
    pack_bins(c, groups);
    const int64_t load = max_bin_load(c);
    int K = c->p.nodes_per_thread;
    int T = c->p.threads_per_group;
    if (K == 0 && T == 0 && split_plan) {
      K = (int)std::min<int64_t>(8, std::max<int64_t>(4, (load + 1023) / 1024));
      T = (int)std::max<int64_t>(64, (load + 64LL * K - 1) / (64LL * K) * 64);
    } else if (K == 0 && T == 0) {
      K = (int)std::min<int64_t>(8, std::max<int64_t>(2, (load + 1023) / 1024));
      T = 64;
      while ((int64_t)T * K < load) T *= 2;
    } else if (K == 0) {
      K = (int)std::max<int64_t>(2, (load + T - 1) / T);
    } else if (T == 0) {
      T = (int)std::max<int64_t>(64, (load + 64LL * K - 1) / (64LL * K) * 64);
    }
    const int maxT = fib::plan_max_threads(K);
    if (maxT > 0 && T <= maxT && (int64_t)T * K >= load) {
      c->K = K;
      c->threads = T;
      c->groups = groups;
      break;
    }
    if (c->p.groups > 0 || groups >= c->n_fibers)
      return fail(FIB_EUNSUPPORTED, "cannot fit %lld nodes into %d bins with the requested shape",
                  (long long)load, groups);
    groups = std::min(groups * 2, c->n_fibers);
  }
  build_tables(c);
  return FIB_OK;
}

// Slot-info words with the stimulus entry of each real slot.
std::vector<uint32_t> slot_info_with_stim(const fib_ctx* c) {
  std::vector<uint32_t> info(c->slot_base);
  if (!c->node_stim.empty())
    for (size_t k = 0; k < info.size(); ++k)
      if (c->slot_gidx[k] >= 0)
        info[k] |= (uint32_t)c->node_stim[c->slot_gidx[k]] << fib::SLOT_STIM_SHIFT;
  return info;
}

// Uploads the slot tables of the current plan (reallocating them if their
// size changed).  The stream must be idle.
int upload_plan(fib_ctx* c, size_t old_slots) {
  const size_t nslots = std::max<size_t>(c->slot_gidx.size(), 1);
  if (nslots != old_slots) {
    (void)hipFree(c->d_slot_gidx);
    (void)hipFree(c->d_slot_info);
    c->d_slot_gidx = nullptr;
    c->d_slot_info = nullptr;
    if (hipMalloc(&c->d_slot_gidx, sizeof(int32_t) * nslots) != hipSuccess ||
        hipMalloc(&c->d_slot_info, sizeof(uint32_t) * nslots) != hipSuccess)
      return fail(FIB_ENOMEM, "device allocation failed");
  }
  const size_t ne = c->ent_s0.size(), nent = c->bin_ent.size() + 3 * ne;
  if (nent != c->ent_alloc) {
    (void)hipFree(c->d_bin_ent);
    c->d_bin_ent = nullptr;
    c->ent_alloc = 0;
    if (hipMalloc(&c->d_bin_ent, sizeof(int32_t) * nent) != hipSuccess)
      return fail(FIB_ENOMEM, "device allocation failed");
    c->ent_alloc = nent;
  }
  {
    std::vector<int32_t> h(c->bin_ent);
    h.insert(h.end(), c->ent_s0.begin(), c->ent_s0.end());
    h.insert(h.end(), c->ent_gofs.begin(), c->ent_gofs.end());
    h.insert(h.end(), c->ent_fiber.begin(), c->ent_fiber.end());
    HIP_TRY(hipMemcpy(c->d_bin_ent, h.data(), sizeof(int32_t) * nent, hipMemcpyHostToDevice));
  }
  const std::vector<uint32_t> info = slot_info_with_stim(c);
  if (!c->slot_gidx.empty()) {
    HIP_TRY(hipMemcpy(c->d_slot_gidx, c->slot_gidx.data(), sizeof(int32_t) * c->slot_gidx.size(),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->d_slot_info, info.data(), sizeof(uint32_t) * info.size(),
                      hipMemcpyHostToDevice));
  }
  return FIB_OK;
}

KArgs base_args(const fib_ctx* c) {
  KArgs a{};
  a.state = c->d_state;
  a.n_total = c->n_total;
  a.slot_gidx = c->d_slot_gidx;
  a.slot_info = c->d_slot_info;
  if (c->d_bin_ent) {
    const size_t nb = c->bin_ent.size(), ne = c->ent_s0.size();
    a.bin_ent = c->d_bin_ent;
    a.ent_s0 = c->d_bin_ent + nb;
    a.ent_gofs = a.ent_s0 + ne;
    a.ent_fiber = a.ent_gofs + ne;
  }
  a.max_ents = c->max_ents;
  a.n_bins = c->groups;
  a.node_stim = c->d_node_stim;
  a.stim = c->d_stim;
  a.t_act = c->d_tact;
  a.v_prev = c->d_vprev;
  a.flag = c->d_flag;
  a.cap = c->cap;
  a.inv_cm = (float)(1.0 / c->p.Cm);
  a.v_th = (float)c->p.v_th;
  a.dt = (float)c->p.dt_split;
  for (int k = 0; k < c->S; ++k) a.rest[k] = (float)c->rest[k];
  return a;
}

int check_ctx(const fib_ctx* c) {
  if (!c) return fail(FIB_EINVAL, "null context");
  return FIB_OK;
}

// Every point of the adaptive computation back to "active" (its initial
// state), as after a new state.
int adapt_reset_points(fib_ctx* c) {
  if (!c->d_pt || c->n_total == 0) return FIB_OK;
  HIP_TRY(hipMemsetAsync(c->d_pt, fib::PT_ACTIVE, 2 * (size_t)c->n_total, c->stream));
  return FIB_OK;
}

// Tables of the adaptive fused kernel for the current plan and stimulus:
// per slot the index of its fiber within the bin, per bin the first
// stimulus step of each fiber.  *ok is false where the kernel cannot take
// the plan (a bin with more than kBinFibers fibers, or not enough LDS).
int adapt_fused_tables(fib_ctx* c, bool* ok) {
  if (c->adapt_tables_plan == c->plan_version && c->adapt_tables_stim == c->stim_version) {
    *ok = c->adapt_fused_ok;
    return FIB_OK;
  }
  *ok = false;
  c->adapt_fused_ok = false;
  c->adapt_tables_plan = c->plan_version;
  c->adapt_tables_stim = c->stim_version;
  const size_t need = fib::lds_bytes_for(c->threads, c->levels) + fib::adapt_lds_extra(c->cap);
  if (need > c->max_lds) return FIB_OK;
  for (auto& b : c->bin_fibers)
    if ((int)b.size() > fib::kBinFibers) return FIB_OK;
  const size_t nslots = (size_t)c->groups * c->cap, nbins = (size_t)c->groups * fib::kBinFibers;
  std::vector<uint8_t> fib_of(std::max<size_t>(nslots, 1), 0);
  std::vector<int32_t> first(std::max<size_t>(nbins, 1), INT32_MAX);
  for (int b = 0; b < c->groups; ++b) {
    size_t pos = (size_t)b * c->cap;
    for (size_t j = 0; j < c->bin_fibers[b].size(); ++j) {
      const int32_t f = c->bin_fibers[b][j];
      first[(size_t)b * fib::kBinFibers + j] = c->first_on[f];
      for (int32_t i = 0; i < c->n_nodes[f]; ++i) fib_of[pos++] = (uint8_t)j;
    }
  }
  if (c->adapt_slots < fib_of.size() || c->adapt_bins < first.size()) {
    (void)hipFree(c->d_slot_fiber);
    (void)hipFree(c->d_bin_first_on);
    c->d_slot_fiber = nullptr;
    c->d_bin_first_on = nullptr;
    c->adapt_slots = c->adapt_bins = 0;
    if (hipMalloc(&c->d_slot_fiber, fib_of.size()) != hipSuccess ||
        hipMalloc(&c->d_bin_first_on, sizeof(int32_t) * first.size()) != hipSuccess) {
      c->adapt_tables_plan = ~0ull;
      return fail(FIB_ENOMEM, "device allocation failed");
    }
    c->adapt_slots = fib_of.size();
    c->adapt_bins = first.size();
  }
  HIP_TRY(hipMemcpy(c->d_slot_fiber, fib_of.data(), fib_of.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->d_bin_first_on, first.data(), sizeof(int32_t) * first.size(),
                    hipMemcpyHostToDevice));
  c->adapt_fused_ok = true;
  *ok = true;
  return FIB_OK;
}

// The point flags of step step0 - 1 must sit in buffer (step0 - 1) & 1.
int adapt_align_flags(fib_ctx* c, int64_t step0) {
  const int want = (int)((step0 + 1) & 1);
  if (want != c->adapt_par)
    HIP_TRY(hipMemcpyAsync(c->d_pt + want * c->n_total, c->d_pt + c->adapt_par * c->n_total,
                           (size_t)c->n_total, hipMemcpyDeviceToDevice, c->stream));
  c->adapt_par = want;
  return FIB_OK;
}

// fib_run with adaptive computation in the fused kernel: one launch; the
// point flags of step0 - 1 in, those of the last step out.
int run_adaptive_fused(fib_ctx* c, KArgs a, int64_t step0, int64_t n_steps) {
  if (int rc = adapt_align_flags(c, step0)) return rc;
  const int64_t end = step0 + n_steps;
  a.pt_prev = c->d_pt + ((step0 + 1) & 1) * c->n_total;
  a.pt_cur = c->d_pt + ((end - 1) & 1) * c->n_total;
  a.adapt_count = c->d_adapt_count;
  a.adapt_tol = (float)c->adapt_tol;
  a.slot_fiber = c->d_slot_fiber;
  a.bin_first_on = c->d_bin_first_on;
  const size_t lds = fib::lds_bytes_for(c->threads, c->levels) + fib::adapt_lds_extra(c->cap);
  HIP_TRY(fib::launch_run_fused_adaptive(c->K, c->groups, c->threads, lds, a, c->stream));
  c->adapt_par = (int)((end - 1) & 1);
  return FIB_OK;
}

// fib_run with adaptive computation (split schedule).  Per Strang step n:
// start(n) [solve set, prescriptions, first half], diffusion(n) [fibers
// with a solved node], finish(n) [second half, check, observables]; per
// Godunov step: start(n) [observables of n-1, solve set, reaction, check],
// diffusion(n), and the observables of the last step after the loop.  The
// point flags of step n live in buffer n & 1, the fiber flags likewise.
int run_adaptive(fib_ctx* c, KArgs a, int64_t step0, int64_t n_steps) {
  const int64_t nt = c->n_total, nf = c->n_fibers;
  const int64_t end = step0 + n_steps;
  const bool godunov = c->p.splitting == FIB_SPLIT_GODUNOV;
  a.node_fiber = c->d_node_fiber;
  a.fiber_first_on = c->d_first_on;
  a.adapt_count = c->d_adapt_count;
  a.adapt_tol = (float)c->adapt_tol;
  auto at = [&](int64_t n) {
    a.pt_cur = c->d_pt + (n & 1) * nt;
    a.pt_prev = c->d_pt + ((n + 1) & 1) * nt;
    a.fiber_any = c->d_fiber_any + (n & 1) * nf;
    a.fiber_any_next = c->d_fiber_any + ((n + 1) & 1) * nf;
  };
  if (int rc = adapt_align_flags(c, step0)) return rc;
  HIP_TRY(hipMemsetAsync(c->d_fiber_any, 0, 2 * (size_t)nf, c->stream));
  HIP_TRY(hipMemcpyAsync(c->d_vprev, c->d_state, sizeof(float) * nt, hipMemcpyDeviceToDevice,
                         c->stream));
  const size_t lds = fib::lds_bytes_for(c->threads, c->levels);
  // ST57: decisions, then the reaction parts over the list of solved nodes
  const bool listed = c->p.model == FIB_MODEL_ST57;
  int32_t* list = c->d_adapt_list;
  int32_t* counts = c->d_adapt_lcount;
  if (listed && (!list || !counts)) return fail(FIB_EINVAL, "adaptive ST57 list not allocated");
  if (listed) HIP_TRY(hipMemsetAsync(counts, 0, 2 * sizeof(int32_t), c->stream));
  auto start = [&](int64_t n, bool godunov_step, bool observe_prev) -> hipError_t {
    if (!listed)
      return fib::launch_adapt_start(c->p.model, godunov_step, (int32_t)n, observe_prev, a,
                                     c->stream);
    const int slot = (int)(n & 1);
    hipError_t e = fib::launch_adapt_decide(godunov_step, (int32_t)n, observe_prev, list, counts,
                                            slot, a, c->stream);
    if (e != hipSuccess) return e;
    return fib::launch_adapt_solve(c->p.model, godunov_step ? 2 : 0, (int32_t)n, list,
                                   counts + slot, a, c->stream);
  };
  // (list form: the observables of step n are taken by the decisions of
  // step n + 1, those of the last step by k_observe)
  auto finish = [&](int64_t n) -> hipError_t {
    if (!listed) return fib::launch_adapt_finish(c->p.model, (int32_t)n, a, c->stream);
    return fib::launch_adapt_solve(c->p.model, 1, (int32_t)n, list, counts + (n & 1), a,
                                   c->stream);
  };
  if (godunov) {
    for (int64_t n = step0; n < end; ++n) {
      at(n);
      HIP_TRY(start(n, true, n > step0));
      HIP_TRY(fib::launch_diffusion(c->K, c->groups, c->threads, lds, a, c->stream));
    }
    KArgs o = a;
    o.fiber_any = nullptr;
    HIP_TRY(fib::launch_react(c->p.model, (int32_t)(end - 1), 0, 2, o, c->stream));
  } else {
    at(step0);
    HIP_TRY(start(step0, false, false));
    for (int64_t n = step0; n < end; ++n) {
      at(n);
      HIP_TRY(fib::launch_diffusion(c->K, c->groups, c->threads, lds, a, c->stream));
      HIP_TRY(finish(n));
      if (n + 1 < end) {
        at(n + 1);
        HIP_TRY(start(n + 1, false, listed));
      }
    }
    if (listed) HIP_TRY(fib::launch_observe((int32_t)(end - 1), a, c->stream));
  }
  c->adapt_par = (int)((end - 1) & 1);
  return FIB_OK;
}

int check_levels_fit(const fib_ctx* c, int levels) {
  const size_t need = fib::lds_bytes_for(c->threads, levels);
  if (need > c->max_lds)
    return fail(FIB_EUNSUPPORTED, "the diffusion solve needs %zu bytes of LDS, the device offers %zu",
                need, c->max_lds);
  return FIB_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

// Kernel timing.  kt_mark() records an event on the context's stream (null
// when timing is off or no event is available); kt_close() files the pair
// (a, b) under a kernel class.  Pairs are read back in order as they
// complete, without blocking, once more than kKtPending are outstanding,
// and all of them by fib_kernel_time.
constexpr size_t kKtPending = 4096;

hipEvent_t kt_mark(fib_ctx* c) {
  if (!c->kt_on) return nullptr;
  hipEvent_t e = nullptr;
  if (!c->kt_pool.empty()) {
    e = c->kt_pool.back();
    c->kt_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return nullptr;
  }
  if (hipEventRecord(e, c->stream) != hipSuccess) {
    c->kt_pool.push_back(e);
    return nullptr;
  }
  return e;
}

void kt_harvest(fib_ctx* c, bool wait) {
  while (!c->kt_pending.empty()) {
    const fib_ctx::KtRec r = c->kt_pending.front();
    if (wait) (void)hipEventSynchronize(r.b);
    float ms = 0.0f;
    const hipError_t e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e == hipErrorNotReady) break;
    if (e == hipSuccess) {
      c->kt_ms[r.cls] += ms;
      c->kt_n[r.cls] += 1;
    }
    if (r.own_a) c->kt_pool.push_back(r.a);
    if (r.own_b) c->kt_pool.push_back(r.b);
    c->kt_pending.pop_front();
  }
}

void kt_close(fib_ctx* c, int cls, hipEvent_t a, hipEvent_t b, bool own_a = true,
              bool own_b = true) {
  if (!a || !b) {
    if (a && own_a) c->kt_pool.push_back(a);
    if (b && own_b) c->kt_pool.push_back(b);
    return;
  }
  c->kt_pending.push_back({cls, a, b, own_a, own_b});
  if (c->kt_pending.size() > kKtPending) kt_harvest(c, false);
}

// A launch between two timing events filed under `cls`.
#define KT_LAUNCH(c, cls, expr)                 \
  do {                                          \
    hipEvent_t kt_a_ = kt_mark(c);              \
    HIP_TRY(expr);                              \
    kt_close((c), (cls), kt_a_, kt_mark(c));    \
  } while (0)

// One surrogate pair (network or closed-form predictor) finishing step n
// and starting step n + 1, with the fallback kernel.
int surrogate_step(fib_ctx* c, const KArgs& a, int64_t n, hipStream_t stream) {
  // the launchers record `mid` between their two kernels (they launch
  // nothing for an empty context); no timing while a graph is captured
  const bool timed = c->kt_on && c->n_total > 0 && stream == c->stream;
  hipEvent_t e0 = timed ? kt_mark(c) : nullptr;
  hipEvent_t mid = nullptr;
  if (timed && !c->kt_pool.empty()) {
    mid = c->kt_pool.back();
    c->kt_pool.pop_back();
  } else if (timed && hipEventCreate(&mid) != hipSuccess) {
    mid = nullptr;
  }
  if (c->sur_pred == FIB_PRED_NETWORK)
    HIP_TRY(fib::launch_surrogate_step(c->p.model, a, c->sur_net, c->d_sur_frags, c->d_sur_bias,
                                       c->d_sur_tab, c->sur_sc, (int32_t)n, c->d_sur_list,
                                       c->d_sur_count, c->sur_slot, c->d_sur_total, c->sur_grid,
                                       mid, stream));
  else
    HIP_TRY(fib::launch_predictor_step(c->p.model, c->sur_pred, a, c->d_sur_tab, (int32_t)n,
                                       c->d_sur_list, c->d_sur_count, c->sur_slot,
                                       c->d_sur_total, c->sur_grid, mid, stream));
  hipEvent_t e1 = timed ? kt_mark(c) : nullptr;
  if (mid && e0 && e1) {
    // the first pair leaves `mid` to the second, which is read back later
    kt_close(c, FIB_KT_SURROGATE, e0, mid, true, false);
    kt_close(c, FIB_KT_FALLBACK, mid, e1, true, true);
  } else {
    kt_close(c, FIB_KT_SURROGATE, e0, nullptr);
    kt_close(c, FIB_KT_SURROGATE, e1, nullptr);
    if (mid) c->kt_pool.push_back(mid);
  }
  c->sur_last_slot = c->sur_slot;
  c->sur_slot ^= 1;
  c->sur_steps += 1;
  return FIB_OK;
}

// ---------------------------------------------------------------------------
// Graph replay of the split schedule.  A block of P consecutive Strang split
// steps -- diffusion, then the reaction pair (or surrogate pair) that ends
// each step and starts the next -- is captured once per fib_run call on a
// non-blocking stream, with the step arguments relative to a device step
// base and a final node that advances the base by P; fib_run then launches
// the executable graph once per block on the context's stream.  Blocks
// start at multiples of P, and P is a multiple of the sample interval, so
// every block writes V_m samples at the same offsets; with a surrogate
// attached it holds an even number of surrogate steps, so the two
// alternating rejection counters end each block where they began.  The
// first and last steps of a call, and steps before the first block, run as
// before.
// ---------------------------------------------------------------------------

// Split steps per graph block for these arguments, or 0 (no replay).
int64_t graph_period(const fib_ctx* c, const KArgs& a) {
  if (!c->graphs || c->kt_on || c->n_total == 0) return 0;
  const int64_t se = a.samples && a.sample_every > 0 ? a.sample_every : 0;
  const int64_t P = se == 0 ? 64 : (se % 2 == 0 ? 2 * se : se);
  return P <= 4096 ? P : 0;
}

// Releases the executable graph of an earlier call once its replays are done.
void graph_release(fib_ctx* c) {
  if (c->graph_done) (void)hipEventSynchronize(c->graph_done);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
}

int surrogate_step(fib_ctx* c, const KArgs& a, int64_t n, hipStream_t stream);

// Captures one block of P steps (relative steps 0 .. P-1) and replays it
// `blocks` times from absolute step n0.
int run_graph_blocks(fib_ctx* c, const KArgs& a, int64_t n0, int64_t P, int64_t blocks) {
  graph_release(c);
  if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  if (!c->graph_done) HIP_TRY(hipEventCreateWithFlags(&c->graph_done, hipEventDisableTiming));
  if (!c->d_step_base && hipMalloc(&c->d_step_base, sizeof(int32_t)) != hipSuccess)
    return fail(FIB_ENOMEM, "device allocation failed");
  KArgs g = a;
  g.step_base = c->d_step_base;
  const size_t lds = fib::lds_bytes_for(c->threads, c->levels);
  const int slot0 = c->sur_slot, last0 = c->sur_last_slot;
  const int64_t steps0 = c->sur_steps;
  HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  int rc = FIB_OK;
  for (int64_t j = 0; j < P && le == hipSuccess && rc == FIB_OK; ++j) {
    le = fib::launch_diffusion(c->K, c->groups, c->threads, lds, g, c->cap_stream);
    if (le != hipSuccess) break;
    const bool sample = g.samples && g.sample_every > 0 && (j + 1) % g.sample_every == 0;
    if (c->sur_on && !sample)
      rc = surrogate_step(c, g, j, c->cap_stream);
    else
      le = fib::launch_react(c->p.model, (int32_t)j, (int32_t)(j + 1), 1 | 2 | 4, g,
                             c->cap_stream);
  }
  if (le == hipSuccess && rc == FIB_OK)
    le = fib::launch_step_base(c->d_step_base, (int32_t)P, false, c->cap_stream);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(c->cap_stream, &graph);
  const int64_t per_block = c->sur_steps - steps0;
  c->sur_steps = steps0;
  if (rc != FIB_OK || le != hipSuccess || ec != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    c->sur_slot = slot0;
    c->sur_last_slot = last0;
    if (rc != FIB_OK) return rc;
    return fail(FIB_EHIP, "graph capture: %s",
                hipGetErrorString(le != hipSuccess ? le : ec));
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(graph);
    c->sur_slot = slot0;
    c->sur_last_slot = last0;
    return fail(FIB_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
  }
  c->graph = graph;
  c->graph_exec = exec;
  // the capture stepped the counter bookkeeping through one block; an even
  // number of surrogate steps leaves the slot where it was
  HIP_TRY(fib::launch_step_base(c->d_step_base, (int32_t)n0, true, c->stream));
  for (int64_t b = 0; b < blocks; ++b) {
    HIP_TRY(hipGraphLaunch(exec, c->stream));
    c->sur_steps += per_block;
    ++c->graph_replays;
  }
  HIP_TRY(hipEventRecord(c->graph_done, c->stream));
  return FIB_OK;
}

// Device buffers of the surrogate step that do not depend on the predictor:
// the rejection list, the two alternating counters (both zero) and the
// running rejection total (zero).
int surrogate_buffers(fib_ctx* c) {
  if (!c->d_sur_tab && hipMalloc(&c->d_sur_tab, sizeof(float) * fib::kSurTabFloats) != hipSuccess)
    return fail(FIB_ENOMEM, "device allocation failed");
  if (!c->d_sur_list) {
    if (hipMalloc(&c->d_sur_list, sizeof(int) * (size_t)std::max<int64_t>(c->n_total, 1)) != hipSuccess ||
        hipMalloc(&c->d_sur_count, 2 * sizeof(int)) != hipSuccess ||
        hipMalloc(&c->d_sur_total, sizeof(unsigned long long)) != hipSuccess)
      return fail(FIB_ENOMEM, "device allocation failed");
  }
  HIP_TRY(hipMemset(c->d_sur_count, 0, 2 * sizeof(int)));
  HIP_TRY(hipMemset(c->d_sur_total, 0, sizeof(unsigned long long)));
  c->sur_slot = 0;
  c->sur_last_slot = -1;
  c->sur_steps = 0;
  return FIB_OK;
}

extern "C" {

const char* fib_last_error(void) { return g_err.c_str(); }

int fib_n_states(int32_t model) {
  const int s = n_states_of(model);
  return s > 0 ? s : fail(FIB_EINVAL, "unknown model %d", model);
}

int fib_check_params(const fib_params* p) {
  if (!p) return fail(FIB_EINVAL, "null parameters");
  if (n_states_of(p->model) <= 0) return fail(FIB_EINVAL, "unknown model %d", p->model);
  if (p->schedule < FIB_SCHED_AUTO || p->schedule > FIB_SCHED_SPLIT)
    return fail(FIB_EINVAL, "unknown schedule %d", p->schedule);
  auto pos = [](double x) { return std::isfinite(x) && x > 0.0; };
  if (!pos(p->Cm) || !pos(p->Am) || !pos(p->h)) return fail(FIB_EINVAL, "Cm, Am and h must be > 0");
  if (!(std::isfinite(p->sigma) && p->sigma >= 0.0)) return fail(FIB_EINVAL, "sigma must be >= 0");
  if (!pos(p->dt_0D) || !pos(p->dt_1D) || !pos(p->dt_split))
    return fail(FIB_EINVAL, "time steps must be > 0");
  if (!std::isfinite(p->v_th)) return fail(FIB_EINVAL, "v_th must be finite");
  if (p->threads_per_group != 0 &&
      (p->threads_per_group % 64 != 0 || p->threads_per_group < 64 || p->threads_per_group > 1024))
    return fail(FIB_EINVAL, "threads_per_group must be 0 or a multiple of 64 in [64, 1024]");
  if (p->nodes_per_thread != 0 && fib::plan_max_threads(p->nodes_per_thread) == 0)
    return fail(FIB_EINVAL, "nodes_per_thread must be 0 or in [2, 14]");
  if (p->threads_per_group != 0 && p->nodes_per_thread != 0 &&
      p->threads_per_group > fib::plan_max_threads(p->nodes_per_thread))
    return fail(FIB_EINVAL, "%d nodes per thread allow at most %d threads per group",
                p->nodes_per_thread, fib::plan_max_threads(p->nodes_per_thread));
  if (p->groups < 0) return fail(FIB_EINVAL, "groups must be >= 0");
  if (p->splitting != FIB_SPLIT_STRANG && p->splitting != FIB_SPLIT_GODUNOV)
    return fail(FIB_EINVAL, "unknown splitting %d", p->splitting);
  if (p->time_1d != FIB_1D_CRANK_NICOLSON && p->time_1d != FIB_1D_IMPLICIT_EULER)
    return fail(FIB_EINVAL, "unknown 1D time stepping %d", p->time_1d);
  if (p->tune != 0 && p->tune != 1) return fail(FIB_EINVAL, "tune must be 0 or 1");
  if (ceil_steps(p->dt_split, p->dt_0D) > (1 << 20) || ceil_steps(p->dt_split, p->dt_1D) > (1 << 20))
    return fail(FIB_EINVAL, "more than 2^20 substeps per split step");
  return FIB_OK;
}

int fib_plan_preview(const fib_params* p, int32_t n_fibers, const int32_t* n_nodes,
                     int32_t compute_units, int32_t* groups, int32_t* threads,
                     int32_t* nodes_per_thread, int32_t* pcr_levels, int64_t* max_load) {
  int rc = fib_check_params(p);
  if (rc) return rc;
  if (n_fibers < 0 || (n_fibers > 0 && !n_nodes) || compute_units < 1)
    return fail(FIB_EINVAL, "bad fiber list or compute-unit count");
  fib_ctx c;
  c.p = *p;
  c.S = n_states_of(p->model);
  c.n_fibers = n_fibers;
  c.n_nodes.assign(n_nodes, n_nodes + n_fibers);
  c.offsets.assign(n_fibers + 1, 0);
  for (int32_t f = 0; f < n_fibers; ++f) {
    if (n_nodes[f] < 1) return fail(FIB_EINVAL, "fiber %d has %d nodes", f, n_nodes[f]);
    c.offsets[f + 1] = c.offsets[f] + n_nodes[f];
  }
  c.n_total = c.offsets[n_fibers];
  c.cu_count = compute_units;
  if ((rc = make_plan(&c))) return rc;
  int64_t mx = 0;
  for (auto& b : c.bin_fibers) {
    int64_t s = 0;
    for (int32_t f : b) s += c.n_nodes[f];
    mx = std::max(mx, s);
  }
  if (groups) *groups = c.groups;
  if (threads) *threads = c.threads;
  if (nodes_per_thread) *nodes_per_thread = c.K;
  if (pcr_levels) *pcr_levels = c.levels;
  if (max_load) *max_load = mx;
  return FIB_OK;
}

int fib_rest_state(const fib_params* p, double* y_out) {
  if (!p || !y_out) return fail(FIB_EINVAL, "null argument");
  if (p->model == FIB_MODEL_HH) return hh_rest(y_out);
  if (p->model == FIB_MODEL_HH_APX_EXP) return hh_rest(y_out, true);
  if (p->model == FIB_MODEL_ST57) return st57_rest(y_out);
  if (p->model == FIB_MODEL_ST57_APX) return st57_rest(y_out, true);
  return fail(FIB_EINVAL, "unknown model %d", p->model);
}

int fib_create(const fib_params* p, int32_t n_fibers, const int32_t* n_nodes, void* stream,
               fib_t** out) {
  if (!out) return fail(FIB_EINVAL, "null output pointer");
  *out = nullptr;
  int rc = fib_check_params(p);
  if (rc) return rc;
  if (n_fibers < 0 || (n_fibers > 0 && !n_nodes)) return fail(FIB_EINVAL, "bad fiber list");
  int64_t total = 0;
  for (int32_t f = 0; f < n_fibers; ++f) {
    if (n_nodes[f] < 1) return fail(FIB_EINVAL, "fiber %d has %d nodes", f, n_nodes[f]);
    total += n_nodes[f];
  }
  if (total >= (int64_t)1 << 31) return fail(FIB_EUNSUPPORTED, "more than 2^31 - 1 nodes");

  fib_ctx* c = new (std::nothrow) fib_ctx();
  if (!c) return fail(FIB_ENOMEM, "host allocation failed");
  c->p = *p;
  c->tune_pending = p->tune != 0;
  c->S = n_states_of(p->model);
  c->n_fibers = n_fibers;
  c->n_nodes.assign(n_nodes, n_nodes + n_fibers);
  c->offsets.assign(n_fibers + 1, 0);
  for (int32_t f = 0; f < n_fibers; ++f) c->offsets[f + 1] = c->offsets[f] + n_nodes[f];
  c->n_total = total;
  c->stream = (hipStream_t)stream;
  c->first_on.assign(n_fibers, INT32_MAX);

  auto bail = [&](int code) {
    fib_destroy(c);
    return code;
  };
  hipDeviceProp_t prop;
  if (hipGetDevice(&c->device) != hipSuccess || hipGetDeviceProperties(&prop, c->device) != hipSuccess)
    return bail(fail(FIB_EHIP, "no HIP device"));
  c->cu_count = prop.multiProcessorCount;
  c->max_lds = prop.sharedMemPerBlock;
  if ((rc = fib_rest_state(p, c->rest))) return bail(rc);
  if ((rc = make_plan(c))) return bail(rc);
  if ((rc = check_levels_fit(c, c->levels))) return bail(rc);
  if (fib::diffusion_lds_bytes(c->threads, c->levels, c->cap, c->max_ents) > c->max_lds)
    return bail(fail(FIB_EUNSUPPORTED,
                     "a bin of %d fibers needs more LDS for the diffusion than the device offers",
                     c->max_ents - 1));

  const size_t nt = (size_t)std::max<int64_t>(total, 1);
  if (hipMalloc(&c->d_state, sizeof(float) * nt * c->S) != hipSuccess ||
      hipMalloc(&c->d_tact, sizeof(float) * nt) != hipSuccess ||
      hipMalloc(&c->d_vprev, sizeof(float) * nt) != hipSuccess ||
      hipMalloc(&c->d_node_stim, sizeof(int32_t) * nt) != hipSuccess ||
      hipMalloc(&c->d_flag, sizeof(int)) != hipSuccess)
    return bail(fail(FIB_ENOMEM, "device allocation failed"));
  if ((rc = upload_plan(c, 0))) return bail(rc);
  if (hipMemset(c->d_node_stim, 0, sizeof(int32_t) * nt) != hipSuccess ||
      hipMemset(c->d_flag, 0, sizeof(int)) != hipSuccess)
    return bail(fail(FIB_EHIP, "device upload failed"));
  if (fib::launch_fill(c->d_tact, total, INFINITY, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return bail(fail(FIB_EHIP, "device initialization failed"));
  *out = c;
  return FIB_OK;
}

void fib_destroy(fib_t* c) {
  if (!c) return;
  if (c->d_state) (void)hipStreamSynchronize(c->stream);
  (void)hipFree(c->d_state);
  (void)hipFree(c->d_tact);
  (void)hipFree(c->d_vprev);
  (void)hipFree(c->d_flag);
  (void)hipFree(c->d_slot_gidx);
  (void)hipFree(c->d_slot_info);
  (void)hipFree(c->d_bin_ent);
  (void)hipFree(c->d_node_stim);
  (void)hipFree(c->d_stim);
  (void)hipFree(c->d_sur_frags);
  (void)hipFree(c->d_sur_bias);
  (void)hipFree(c->d_sur_tab);
  (void)hipFree(c->d_sur_list);
  (void)hipFree(c->d_sur_count);
  (void)hipFree(c->d_sur_total);
  (void)hipFree(c->d_node_fiber);
  (void)hipFree(c->d_first_on);
  (void)hipFree(c->d_pt);
  (void)hipFree(c->d_fiber_any);
  (void)hipFree(c->d_adapt_count);
  (void)hipFree(c->d_adapt_list);
  (void)hipFree(c->d_adapt_lcount);
  (void)hipFree(c->d_slot_fiber);
  (void)hipFree(c->d_bin_first_on);
  for (const auto& r : c->kt_pending) {
    if (r.own_a) (void)hipEventDestroy(r.a);
    if (r.own_b) (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : c->kt_pool) (void)hipEventDestroy(e);
  graph_release(c);
  if (c->graph_done) (void)hipEventDestroy(c->graph_done);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  (void)hipFree(c->d_step_base);
  delete c;
}

int64_t fib_n_total(const fib_t* c) { return c ? c->n_total : 0; }

int fib_plan_info(const fib_t* c, int32_t* groups, int32_t* threads, int32_t* nodes_per_thread,
                  int32_t* pcr_levels) {
  if (int rc = check_ctx(c)) return rc;
  if (groups) *groups = c->groups;
  if (threads) *threads = c->threads;
  if (nodes_per_thread) *nodes_per_thread = c->K;
  if (pcr_levels) *pcr_levels = c->levels;
  return FIB_OK;
}

int fib_state_device(fib_t* c, float** state, double* ref) {
  if (int rc = check_ctx(c)) return rc;
  if (!state) return fail(FIB_EINVAL, "null output pointer");
  *state = c->d_state;
  if (ref)
    for (int k = 0; k < c->S; ++k) ref[k] = (double)(float)c->rest[k];
  return FIB_OK;
}

int fib_init_state(fib_t* c, const float* vm_noise, const float* rel_noise) {
  if (int rc = check_ctx(c)) return rc;
  KArgs a = base_args(c);
  HIP_TRY(hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream));
  HIP_TRY(fib::launch_init(c->p.model, vm_noise, rel_noise, a, c->stream));
  if (int rc = adapt_reset_points(c)) return rc;
  c->state_ready = true;
  return FIB_OK;
}

int fib_set_state(fib_t* c, const double* y, int64_t n_values) {
  if (int rc = check_ctx(c)) return rc;
  if (n_values != (int64_t)c->S * c->n_total) return fail(FIB_EINVAL, "expected %lld values",
                                                          (long long)c->S * c->n_total);
  if (n_values == 0) { c->state_ready = true; return FIB_OK; }
  if (!y) return fail(FIB_EINVAL, "null state");
  std::vector<float> f(n_values);
  for (int64_t i = 0; i < n_values; ++i) f[i] = (float)(y[i] - (double)(float)c->rest[i / std::max<int64_t>(c->n_total, 1)]);
  HIP_TRY(hipMemcpyAsync(c->d_state, f.data(), sizeof(float) * n_values, hipMemcpyHostToDevice,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(c->d_vprev, c->d_state, sizeof(float) * c->n_total,
                         hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream));
  if (int rc = adapt_reset_points(c)) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->state_ready = true;
  return FIB_OK;
}

int fib_get_state(fib_t* c, double* y, int64_t n_values) {
  if (int rc = check_ctx(c)) return rc;
  if (n_values != (int64_t)c->S * c->n_total) return fail(FIB_EINVAL, "expected %lld values",
                                                          (long long)c->S * c->n_total);
  if (n_values == 0) return FIB_OK;
  if (!y) return fail(FIB_EINVAL, "null output");
  std::vector<float> f(n_values);
  HIP_TRY(hipMemcpyAsync(f.data(), c->d_state, sizeof(float) * n_values, hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  bool bad = false;
  for (int64_t i = 0; i < n_values; ++i) {
    y[i] = (double)f[i] + (double)(float)c->rest[i / c->n_total];
    bad |= !std::isfinite(f[i]);
  }
  if (bad) return fail(FIB_ENONFINITE, "the state holds non-finite values");
  return FIB_OK;
}

int fib_set_stimulus(fib_t* c, const fib_stim* s, int32_t n) {
  if (int rc = check_ctx(c)) return rc;
  if (n < 0 || (n > 0 && !s)) return fail(FIB_EINVAL, "bad stimulus table");
  std::vector<int32_t> node_stim(c->n_total, 0);
  std::vector<fib::StimDev> tab(n);
  std::vector<int32_t> first_on(c->n_fibers, INT32_MAX);
  const int64_t lim = ((int64_t)1 << 31) - 1;
  for (int32_t e = 0; e < n; ++e) {
    const fib_stim& x = s[e];
    if (x.fiber < 0 || x.fiber >= c->n_fibers) return fail(FIB_EINVAL, "entry %d: bad fiber", e);
    if (x.half_width < 0) return fail(FIB_EINVAL, "entry %d: negative half width", e);
    if (x.step_on < 0 || x.step_on > lim || x.n_steps < 0 || x.n_steps > lim || x.period < 0 ||
        x.period > lim)
      return fail(FIB_EINVAL, "entry %d: step indices must lie in [0, 2^31)", e);
    if (!std::isfinite(x.amp)) return fail(FIB_EINVAL, "entry %d: non-finite amplitude", e);
    if (x.mode != FIB_STIM_CURRENT && x.mode != FIB_STIM_VOLTAGE)
      return fail(FIB_EINVAL, "entry %d: unknown mode %d", e, x.mode);
    // voltage entries hold the prescribed value as the device state does:
    // the offset from the resting V_m
    const bool volt = x.mode == FIB_STIM_VOLTAGE;
    if (x.n_steps > 0) first_on[x.fiber] = std::min(first_on[x.fiber], (int32_t)x.step_on);
    tab[e] = fib::StimDev{(int32_t)x.step_on, (int32_t)x.n_steps, (int32_t)x.period,
                          (float)(volt ? x.amp - (double)(float)c->rest[0] : x.amp), volt ? 1 : 0};
    const int64_t n_f = c->n_nodes[x.fiber];
    for (int64_t j = (int64_t)x.node - x.half_width; j <= (int64_t)x.node + x.half_width; ++j) {
      if (j < 0 || j >= n_f) continue;
      int32_t& slot = node_stim[c->offsets[x.fiber] + j];
      if (slot != 0) return fail(FIB_EINVAL, "entry %d: node %lld of fiber %d already stimulated",
                                 e, (long long)j, x.fiber);
      slot = e + 1;
    }
  }
  if ((int64_t)n + 1 >= ((int64_t)1 << (32 - fib::SLOT_STIM_SHIFT)))
    return fail(FIB_EINVAL, "too many stimulus entries");
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->node_stim = node_stim;
  const std::vector<uint32_t> info = slot_info_with_stim(c);
  (void)hipFree(c->d_stim);
  c->d_stim = nullptr;
  c->n_stim = 0;
  if (n > 0) {
    if (hipMalloc(&c->d_stim, sizeof(fib::StimDev) * n) != hipSuccess)
      return fail(FIB_ENOMEM, "device allocation failed");
    HIP_TRY(hipMemcpy(c->d_stim, tab.data(), sizeof(fib::StimDev) * n, hipMemcpyHostToDevice));
  }
  c->n_stim = n;
  c->first_on = first_on;
  ++c->stim_version;
  if (c->d_first_on && c->n_fibers > 0)
    HIP_TRY(hipMemcpy(c->d_first_on, first_on.data(), sizeof(int32_t) * c->n_fibers,
                      hipMemcpyHostToDevice));
  if (c->n_total > 0)
    HIP_TRY(hipMemcpy(c->d_node_stim, node_stim.data(), sizeof(int32_t) * c->n_total,
                      hipMemcpyHostToDevice));
  if (!info.empty())
    HIP_TRY(hipMemcpy(c->d_slot_info, info.data(), sizeof(uint32_t) * info.size(),
                      hipMemcpyHostToDevice));
  return FIB_OK;
}

int fib_step_reaction(fib_t* c, int64_t step, double span) {
  if (int rc = check_ctx(c)) return rc;
  if (!(std::isfinite(span) && span > 0.0)) return fail(FIB_EINVAL, "span must be > 0");
  if (step < 0 || step >= ((int64_t)1 << 31)) return fail(FIB_EINVAL, "step out of range");
  if (!c->state_ready) return fail(FIB_ESTATE, "state not initialized");
  KArgs a = base_args(c);
  const int64_t ns = ceil_steps(span, c->p.dt_0D);
  if (ns > (1 << 20)) return fail(FIB_EINVAL, "more than 2^20 substeps");
  a.n_sub = (int32_t)ns;
  a.tau = (float)(span / (double)ns);
  HIP_TRY(fib::launch_react(c->p.model, (int32_t)step, 0, 1, a, c->stream));
  return FIB_OK;
}

int fib_state_rows(fib_t* c, float* U) {
  if (int rc = check_ctx(c)) return rc;
  if (!c->state_ready) return fail(FIB_ESTATE, "state not initialized");
  if (!U && c->n_total > 0) return fail(FIB_EINVAL, "U is null");
  HIP_TRY(fib::launch_state_rows(c->d_state, c->n_total, c->S, U, c->stream));
  return FIB_OK;
}

int fib_reaction_increments(fib_t* c, const float* U, int64_t rows, int64_t step, float* dU) {
  if (int rc = check_ctx(c)) return rc;
  if (rows < 0 || (rows > 0 && (!U || !dU))) return fail(FIB_EINVAL, "bad arguments");
  if (step < 0 || step >= ((int64_t)1 << 31)) return fail(FIB_EINVAL, "step out of range");
  if (rows == 0) return FIB_OK;
  if (c->n_total == 0) return fail(FIB_EINVAL, "the context has no nodes");
  KArgs a = base_args(c);
  const double span = 0.5 * c->p.dt_split;
  const int64_t ns = ceil_steps(span, c->p.dt_0D);
  if (ns > (1 << 20)) return fail(FIB_EINVAL, "more than 2^20 substeps");
  a.n_sub = (int32_t)ns;
  a.tau = (float)(span / (double)ns);
  const int64_t nt = c->n_total;
  for (int64_t r0 = 0; r0 < rows; r0 += nt) {
    const int64_t n = std::min<int64_t>(nt, rows - r0);
    HIP_TRY(fib::launch_rows_to_state(U, r0, n, c->S, c->d_state, nt, c->stream));
    HIP_TRY(fib::launch_react(c->p.model, (int32_t)step, 0, 1, a, c->stream));
    HIP_TRY(fib::launch_react(c->p.model, (int32_t)step, 0, 1, a, c->stream));
    HIP_TRY(fib::launch_state_minus_rows(c->d_state, U, r0, n, c->S, nt, dU, c->stream));
  }
  c->state_ready = true;
  return FIB_OK;
}

int fib_step_diffusion(fib_t* c, double span) {
  if (int rc = check_ctx(c)) return rc;
  if (!(std::isfinite(span) && span > 0.0)) return fail(FIB_EINVAL, "span must be > 0");
  if (!c->state_ready) return fail(FIB_ESTATE, "state not initialized");
  if (c->n_total == 0) return FIB_OK;
  KArgs a = base_args(c);
  const int64_t m = ceil_steps(span, c->p.dt_1D);
  if (m > (1 << 20)) return fail(FIB_EINVAL, "more than 2^20 substeps");
  a.n_cn = (int32_t)m;
  set_diffusion(c, span / (double)m, a);
  const double r_mat = 2.0 * theta_of(c->p) * cn_r(c, span / (double)m);
  if (c->lv_cache_version != c->plan_version || c->lv_cache_r != r_mat) {
    c->lv_cache_levels = max_pcr_levels(c, r_mat);
    c->lv_cache_r = r_mat;
    c->lv_cache_version = c->plan_version;
  }
  const int lv = c->lv_cache_levels;
  if (int rc = check_levels_fit(c, lv)) return rc;
  a.pcr_levels = lv;
  KT_LAUNCH(c, FIB_KT_DIFFUSION,
            fib::launch_diffusion(c->K, c->groups, c->threads, fib::lds_bytes_for(c->threads, lv),
                                  a, c->stream));
  return FIB_OK;
}

int fib_run(fib_t* c, int64_t step0, int64_t n_steps, int64_t sample_every, float* samples,
            int64_t sample_rows) {
  if (int rc = check_ctx(c)) return rc;
  const int64_t lim = ((int64_t)1 << 31) - 1;
  if (step0 < 0 || n_steps < 0 || step0 + n_steps > lim)
    return fail(FIB_EINVAL, "steps must lie in [0, 2^31)");
  if (sample_every < 0) return fail(FIB_EINVAL, "sample_every must be >= 0");
  if (!c->state_ready) return fail(FIB_ESTATE, "state not initialized");
  if (n_steps == 0 || c->n_total == 0) return FIB_OK;
  if (c->tune_pending) {
    c->tune_pending = false;  // first: the autotuner's trials run fib_run themselves
    if (int rc = fib_autotune(c, 100, 8, nullptr)) return rc;
  }
  KArgs a = base_args(c);
  if (samples && sample_every > 0) {
    const int64_t rows = (step0 + n_steps) / sample_every - step0 / sample_every;
    if (sample_rows < rows) return fail(FIB_EINVAL, "samples holds %lld rows, %lld needed",
                                        (long long)sample_rows, (long long)rows);
    a.samples = samples;
    a.sample_every = sample_every;
    a.sample_row0 = step0 / sample_every;
    a.sample_rows = sample_rows;
  }
  // reaction span before the diffusion: half a split step (Strang) or the
  // whole step (Godunov)
  const bool godunov = c->p.splitting == FIB_SPLIT_GODUNOV;
  const double span = godunov ? c->p.dt_split : 0.5 * c->p.dt_split;
  const int64_t ns = ceil_steps(span, c->p.dt_0D);
  const int64_t nc = ceil_steps(c->p.dt_split, c->p.dt_1D);
  a.n_sub = (int32_t)ns;
  a.n_sub2 = godunov ? 0 : (int32_t)ns;
  a.tau = (float)(span / (double)ns);
  a.n_cn = (int32_t)nc;
  set_diffusion(c, c->p.dt_split / (double)nc, a);
  a.pcr_levels = c->levels;
  a.step0 = (int32_t)step0;
  a.n_steps = (int32_t)n_steps;
  if (c->adapt_tol > 0.0) {
    // fused where the model and the plan allow it, else split
    const bool want_fused = c->p.schedule == FIB_SCHED_FUSED ||
                            (c->p.schedule == FIB_SCHED_AUTO && c->p.model == FIB_MODEL_HH);
    if (c->p.schedule == FIB_SCHED_FUSED && c->p.model == FIB_MODEL_HH_APX_EXP)
      return fail(FIB_EUNSUPPORTED, "the adaptive fused kernel holds the exact Hodgkin-Huxley "
                  "membrane only");
    if (want_fused) {
      if (c->p.model != FIB_MODEL_HH)
        return fail(FIB_EUNSUPPORTED, "the fused schedule holds Hodgkin-Huxley states only");
      bool ok = false;
      if (int rc = adapt_fused_tables(c, &ok)) return rc;
      if (ok) return run_adaptive_fused(c, a, step0, n_steps);
      if (c->p.schedule == FIB_SCHED_FUSED)
        return fail(FIB_EUNSUPPORTED, "the plan does not fit the adaptive fused kernel (at most "
                    "%d fibers per bin, its states in LDS)", fib::kBinFibers);
    }
    return run_adaptive(c, a, step0, n_steps);
  }
  // AUTO: fused for Hodgkin-Huxley unless a surrogate is attached (the
  // surrogate step belongs to the split schedule)
  const bool hh_like = c->p.model == FIB_MODEL_HH || c->p.model == FIB_MODEL_HH_APX_EXP;
  const bool fused = c->p.schedule == FIB_SCHED_FUSED ||
                     (c->p.schedule == FIB_SCHED_AUTO && hh_like && !c->sur_on);
  if (fused) {
    if (!hh_like)
      return fail(FIB_EUNSUPPORTED, "the fused schedule holds Hodgkin-Huxley states only");
    KT_LAUNCH(c, FIB_KT_FUSED,
              fib::launch_run_fused(c->p.model, c->K, c->groups, c->threads,
                                    fib::lds_bytes_for(c->threads, c->levels), a, c->stream));
    return FIB_OK;
  }
  HIP_TRY(hipMemcpyAsync(c->d_vprev, c->d_state, sizeof(float) * c->n_total,
                         hipMemcpyDeviceToDevice, c->stream));
  const size_t lds = fib::lds_bytes_for(c->threads, c->levels);
  const int64_t end = step0 + n_steps;
  if (godunov) {
    // SPLIT, Godunov: per split step one reaction launch (observables of
    // step n-1, then step n's prescriptions and its whole reaction) and one
    // diffusion launch; the observables of the last step follow the loop
    for (int64_t n = step0; n < end; ++n) {
      const int flags = (n > step0 ? 2 : 0) | 4;
      KT_LAUNCH(c, FIB_KT_REACTION,
                fib::launch_react(c->p.model, (int32_t)(n - 1), (int32_t)n, flags, a, c->stream));
      KT_LAUNCH(c, FIB_KT_DIFFUSION,
                fib::launch_diffusion(c->K, c->groups, c->threads, lds, a, c->stream));
    }
    KT_LAUNCH(c, FIB_KT_REACTION,
              fib::launch_react(c->p.model, (int32_t)(end - 1), 0, 2, a, c->stream));
    return FIB_OK;
  }
  // SPLIT, Strang: per split step one diffusion launch and one reaction
  // launch that finishes step n (second half, observables) and starts step
  // n+1 (prescriptions, first half); whole blocks of steps as graph replays
  KT_LAUNCH(c, FIB_KT_REACTION, fib::launch_react(c->p.model, 0, (int32_t)step0, 4, a, c->stream));
  auto eager = [&](int64_t n) -> int {
    KT_LAUNCH(c, FIB_KT_DIFFUSION,
              fib::launch_diffusion(c->K, c->groups, c->threads, lds, a, c->stream));
    const bool last = n + 1 >= end;
    const bool sample = a.samples && a.sample_every > 0 && (n + 1) % a.sample_every == 0;
    if (c->sur_on && !last && !sample) {
      if (int rc = surrogate_step(c, a, n, c->stream)) return rc;
    } else {
      const int flags = 1 | 2 | (last ? 0 : 4);
      KT_LAUNCH(c, FIB_KT_REACTION,
                fib::launch_react(c->p.model, (int32_t)n, (int32_t)(n + 1), flags, a, c->stream));
    }
    return FIB_OK;
  };
  int64_t n = step0;
  const int64_t P = graph_period(c, a);
  if (P > 0) {
    for (; n < end && n % P != 0; ++n)
      if (int rc = eager(n)) return rc;
    // whole blocks, none of which holds the last step of the call
    const int64_t blocks = n < end ? (end - 1 - n) / P : 0;
    if (blocks > 0) {
      if (int rc = run_graph_blocks(c, a, n, P, blocks)) return rc;
      n += blocks * P;
    }
  }
  for (; n < end; ++n)
    if (int rc = eager(n)) return rc;
  return FIB_OK;
}

static int autotune_impl(fib_t* c, int32_t trial_steps, int32_t max_candidates, double* ms_per_step);

int fib_autotune(fib_t* c, int32_t trial_steps, int32_t max_candidates, double* ms_per_step) {
  if (int rc = check_ctx(c)) return rc;
  // the trials time the plain schedule; the adaptive flags stay untouched
  const double tol = c->adapt_tol;
  c->adapt_tol = 0.0;
  const int rc = autotune_impl(c, trial_steps, max_candidates, ms_per_step);
  c->adapt_tol = tol;
  return rc;
}

static int autotune_impl(fib_t* c, int32_t trial_steps, int32_t max_candidates, double* ms_per_step) {
  if (trial_steps < 1 || trial_steps > 100000) return fail(FIB_EINVAL, "trial_steps must be in [1, 100000]");
  if (max_candidates < 1) return fail(FIB_EINVAL, "max_candidates must be >= 1");
  if (!c->state_ready) return fail(FIB_ESTATE, "state not initialized");
  if (ms_per_step) *ms_per_step = 0.0;
  if (c->n_total == 0) return FIB_OK;
  // candidate shapes for the current bins: every workgroup size (multiple of
  // 64) and nodes per thread that hold the heaviest bin with at most 30 %
  // padding, ranked by the slots one SIMD sweeps per step (waves per SIMD x K)
  const int64_t load = max_bin_load(c);
  struct Cand { int T, K; int64_t cost; };
  std::vector<Cand> cand;
  for (int K = 2; K <= 14; ++K) {
    const int maxT = fib::plan_max_threads(K);
    for (int T = 64; T <= maxT; T += 64) {
      const int64_t capn = (int64_t)T * K;
      if (capn < load || capn * 10 > load * 13) continue;
      if (fib::lds_bytes_for(T, 1) > c->max_lds) continue;
      cand.push_back({T, K, (int64_t)((T / 64 + 3) / 4) * K});
    }
  }
  std::sort(cand.begin(), cand.end(), [](const Cand& x, const Cand& y) {
    return x.cost != y.cost ? x.cost < y.cost : x.T < y.T;
  });
  std::vector<Cand> trial;
  trial.push_back({c->threads, c->K, 0});
  for (const Cand& x : cand) {
    if ((int)trial.size() >= max_candidates) break;
    if (x.cost * 100 > cand[0].cost * 112) break;
    if (x.T == c->threads && x.K == c->K) continue;
    trial.push_back(x);
  }
  // the trial runs start from the current state and observables; keep copies
  HIP_TRY(hipStreamSynchronize(c->stream));
  const size_t sb = sizeof(float) * (size_t)c->n_total * c->S, ob = sizeof(float) * (size_t)c->n_total;
  float *s_state = nullptr, *s_tact = nullptr, *s_vprev = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    (void)hipFree(s_state);
    (void)hipFree(s_tact);
    (void)hipFree(s_vprev);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipMalloc(&s_state, sb) != hipSuccess || hipMalloc(&s_tact, ob) != hipSuccess ||
      hipMalloc(&s_vprev, ob) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(FIB_ENOMEM, "autotune: scratch allocation failed");
  }
  auto copy_all = [&](bool save) -> hipError_t {
    hipError_t e = hipMemcpyAsync(save ? s_state : c->d_state, save ? c->d_state : s_state, sb,
                                  hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(save ? s_tact : c->d_tact, save ? c->d_tact : s_tact, ob,
                         hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(save ? s_vprev : c->d_vprev, save ? c->d_vprev : s_vprev, ob,
                         hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e;
  };
  int rc = FIB_OK;
  if (copy_all(true) != hipSuccess) rc = fail(FIB_EHIP, "autotune: state copy failed");
  double best = -1.0;
  Cand pick = trial[0];
  for (const Cand& x : trial) {
    if (rc) break;
    const size_t old = std::max<size_t>(c->slot_gidx.size(), 1);
    c->threads = x.T;
    c->K = x.K;
    build_tables(c);
    if (fib::lds_bytes_for(c->threads, c->levels) > c->max_lds) continue;
    if ((rc = upload_plan(c, old))) break;
    if (copy_all(false) != hipSuccess) { rc = fail(FIB_EHIP, "autotune: state copy failed"); break; }
    if ((rc = fib_run(c, 0, 1, 0, nullptr, 0))) break;  // warm-up (code object load)
    if (copy_all(false) != hipSuccess) { rc = fail(FIB_EHIP, "autotune: state copy failed"); break; }
    if (hipEventRecord(e0, c->stream) != hipSuccess) { rc = fail(FIB_EHIP, "autotune: event failed"); break; }
    if ((rc = fib_run(c, 0, trial_steps, 0, nullptr, 0))) break;
    float ms = 0.0f;
    if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = fail(FIB_EHIP, "autotune: timing failed");
      break;
    }
    if (best < 0.0 || ms < best) {
      best = ms;
      pick = x;
    }
  }
  // the chosen shape, and the state and observables as before
  if (!rc) {
    const size_t old = std::max<size_t>(c->slot_gidx.size(), 1);
    c->threads = pick.T;
    c->K = pick.K;
    build_tables(c);
    rc = upload_plan(c, old);
  }
  if (copy_all(false) != hipSuccess && !rc) rc = fail(FIB_EHIP, "autotune: state copy failed");
  cleanup();
  if (!rc && ms_per_step) *ms_per_step = best / trial_steps;
  return rc;
}

int fib_set_surrogate(fib_t* c, const fib_mlp_t* net, const float* in_shift, const float* in_scale,
                      const float* out_shift, const float* out_scale, const float* res_scale,
                      double flag_scale, double tol) {
  if (int rc = check_ctx(c)) return rc;
  if (!net || !in_shift || !in_scale || !out_shift || !out_scale || !res_scale)
    return fail(FIB_EINVAL, "null argument");
  if (!(tol > 0.0) || !std::isfinite(flag_scale)) return fail(FIB_EINVAL, "bad tolerance or flag scale");
  if (c->p.splitting != FIB_SPLIT_STRANG)
    return fail(FIB_EUNSUPPORTED, "the surrogate step replaces Strang reaction halves");
  if (c->adapt_tol > 0.0)
    return fail(FIB_EUNSUPPORTED, "adaptive computation and the surrogate step do not combine");
  const fib::MlpShape& ms = fib::mlp_shape(net);
  const int S = c->S;
  // supported shapes: the kernels are compiled for them
  bool ok = false;
  if (c->p.model == FIB_MODEL_HH)
    ok = ms.L == 4 && (ms.size[0] == 4 || ms.size[0] == 5) && ms.size[1] == 64 &&
         ms.size[2] == 64 && ms.size[3] == 64 && ms.size[4] == 4;
  else if (c->p.model == FIB_MODEL_ST57)
    ok = ms.L == 3 && (ms.size[0] == 57 || ms.size[0] == 58) && ms.size[1] == 128 &&
         ms.size[2] == 128 && ms.size[3] == 57;
  if (!ok)
    return fail(FIB_EUNSUPPORTED, "surrogate shape not supported for this model (Hodgkin-Huxley: "
                "4 or 5 -> 64 -> 64 -> 64 -> 4; ST57: 57 or 58 -> 128 -> 128 -> 57)");
  fib::SurrogateNet sn{};
  sn.L = ms.L;
  sn.act = ms.act;
  int frags = 0, bias = 0;
  for (int l = 1; l <= ms.L; ++l) {
    sn.n_in[l] = ms.size[l - 1];
    sn.n_out[l] = ms.size[l];
    sn.pad_in[l] = (ms.size[l - 1] + 31) / 32 * 32;
    sn.pad_out[l] = (ms.size[l] + 15) / 16 * 16;
    sn.w_off[l] = ms.w_off[l];
    sn.b_off[l] = ms.b_off[l];
    sn.frag_off[l] = frags;
    frags += (sn.pad_out[l] / 16) * (sn.pad_in[l] / 32);
    sn.bias_off[l] = bias;
    bias += sn.pad_out[l];
  }
  sn.frag_off[ms.L + 1] = frags;
  sn.bias_off[ms.L + 1] = bias;
  sn.frag_elems = (int64_t)frags * 512;
  sn.bias_elems = bias;
  fib::SurrogateScales sc{};
  sc.n_in = ms.size[0];
  sc.flag_scale = (float)flag_scale;
  sc.tol = (float)tol;
  std::vector<float> tab((size_t)fib::kSurTabFloats, 0.0f);
  const KArgs a0 = base_args(c);
  for (int k = 0; k < S; ++k) {
    if (!(in_scale[k] > 0.0f) || !(out_scale[k] > 0.0f) || !(res_scale[k] > 0.0f) ||
        !std::isfinite(in_shift[k]) || !std::isfinite(out_shift[k]) ||
        !std::isfinite(in_scale[k]) || !std::isfinite(out_scale[k]) || !std::isfinite(res_scale[k]))
      return fail(FIB_EINVAL, "state %d: scales must be finite and > 0", k);
    tab[fib::kTabIn + 2 * k] = in_scale[k];
    tab[fib::kTabIn + 2 * k + 1] = -in_shift[k] * in_scale[k];
    tab[fib::kTabMid + 2 * k] = 0.5f * out_scale[k];
    tab[fib::kTabMid + 2 * k + 1] = 0.5f * out_shift[k] + a0.rest[k];
    tab[fib::kTabChk + 4 * k] = out_scale[k];
    tab[fib::kTabChk + 4 * k + 1] = out_shift[k];
    tab[fib::kTabChk + 4 * k + 2] = (float)(tol * (double)res_scale[k]);
    tab[fib::kTabChk + 4 * k + 3] = a0.rest[k];
  }
  const size_t lds = fib::surrogate_lds_bytes(c->p.model, sn);
  if (lds > c->max_lds) return fail(FIB_EUNSUPPORTED, "surrogate needs %zu bytes of LDS", lds);
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipStreamSynchronize(fib::mlp_stream(net)));
  (void)hipFree(c->d_sur_frags);
  (void)hipFree(c->d_sur_bias);
  c->d_sur_frags = nullptr;
  c->d_sur_bias = nullptr;
  c->sur_on = false;
  if (hipMalloc(&c->d_sur_frags, (size_t)sn.frag_elems * 2) != hipSuccess ||
      hipMalloc(&c->d_sur_bias, (size_t)sn.bias_elems * 4) != hipSuccess)
    return fail(FIB_ENOMEM, "device allocation failed");
  // both rejection counters start at zero; each surrogate step clears the
  // one the next step uses
  if (int rc = surrogate_buffers(c)) return rc;
  HIP_TRY(hipMemcpy(c->d_sur_tab, tab.data(), sizeof(float) * tab.size(), hipMemcpyHostToDevice));
  HIP_TRY(fib::launch_pack(sn, fib::mlp_device_params(net), c->d_sur_frags, c->d_sur_bias, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(4, c->max_lds / lds));
  c->sur_grid = c->cu_count * per_cu;
  c->sur_net = sn;
  c->sur_sc = sc;
  c->sur_pred = FIB_PRED_NETWORK;
  c->sur_on = true;
  return FIB_OK;
}

int fib_set_predictor(fib_t* c, int32_t predictor, const float* res_scale, double tol) {
  if (int rc = check_ctx(c)) return rc;
  if (predictor != FIB_PRED_ZERO && predictor != FIB_PRED_EULER)
    return fail(FIB_EINVAL, "unknown predictor %d", predictor);
  if (!res_scale) return fail(FIB_EINVAL, "null argument");
  if (!(tol > 0.0)) return fail(FIB_EINVAL, "bad tolerance");
  if (c->p.splitting != FIB_SPLIT_STRANG)
    return fail(FIB_EUNSUPPORTED, "the surrogate step replaces Strang reaction halves");
  if (c->adapt_tol > 0.0)
    return fail(FIB_EUNSUPPORTED, "adaptive computation and the surrogate step do not combine");
  if (c->p.model != FIB_MODEL_HH && c->p.model != FIB_MODEL_ST57)
    return fail(FIB_EUNSUPPORTED, "the surrogate step holds Hodgkin-Huxley and ST57");
  const KArgs a0 = base_args(c);
  std::vector<float> tab((size_t)fib::kSurTabFloats, 0.0f);
  for (int k = 0; k < c->S; ++k) {
    if (!(res_scale[k] > 0.0f) || !std::isfinite(res_scale[k]))
      return fail(FIB_EINVAL, "state %d: res_scale must be finite and > 0", k);
    tab[fib::kTabChk + 4 * k + 2] = (float)(tol * (double)res_scale[k]);
    tab[fib::kTabChk + 4 * k + 3] = a0.rest[k];
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->sur_on = false;
  if (int rc = surrogate_buffers(c)) return rc;
  HIP_TRY(hipMemcpy(c->d_sur_tab, tab.data(), sizeof(float) * tab.size(), hipMemcpyHostToDevice));
  c->sur_grid = c->cu_count * 8;
  c->sur_pred = predictor;
  c->sur_on = true;
  return FIB_OK;
}

int fib_step_surrogate(fib_t* c, int64_t step) {
  if (int rc = check_ctx(c)) return rc;
  if (!c->sur_on) return fail(FIB_ESTATE, "no surrogate attached");
  if (!c->state_ready) return fail(FIB_ESTATE, "state not initialized");
  if (step < 0 || step + 1 >= ((int64_t)1 << 31)) return fail(FIB_EINVAL, "step out of range");
  KArgs a = base_args(c);
  const int64_t ns = ceil_steps(0.5 * c->p.dt_split, c->p.dt_0D);
  a.n_sub = (int32_t)ns;
  a.tau = (float)(0.5 * c->p.dt_split / (double)ns);
  return surrogate_step(c, a, step, c->stream);
}

int fib_surrogate_predict(fib_t* c, int64_t step, float* du) {
  if (int rc = check_ctx(c)) return rc;
  if (!c->sur_on) return fail(FIB_ESTATE, "no surrogate attached");
  if (c->sur_pred != FIB_PRED_NETWORK)
    return fail(FIB_ESTATE, "the attached step has a closed-form predictor, not a network");
  if (!c->state_ready) return fail(FIB_ESTATE, "state not initialized");
  if (!du && c->n_total > 0) return fail(FIB_EINVAL, "du is null");
  if (step < 0 || step + 1 >= ((int64_t)1 << 31)) return fail(FIB_EINVAL, "step out of range");
  KArgs a = base_args(c);
  HIP_TRY(fib::launch_surrogate_predict(c->p.model, a, c->sur_net, c->d_sur_frags, c->d_sur_bias,
                                        c->d_sur_tab, c->sur_sc, (int32_t)step, du, c->sur_grid,
                                        c->stream));
  return FIB_OK;
}

int fib_clear_surrogate(fib_t* c) {
  if (int rc = check_ctx(c)) return rc;
  c->sur_on = false;
  return FIB_OK;
}

int fib_surrogate_last_fallbacks(fib_t* c, int64_t* n) {
  if (int rc = check_ctx(c)) return rc;
  if (!n) return fail(FIB_EINVAL, "null output");
  *n = 0;
  if (!c->d_sur_count || c->sur_last_slot < 0) return FIB_OK;
  int v = 0;
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(&v, c->d_sur_count + c->sur_last_slot, sizeof(int), hipMemcpyDeviceToHost));
  *n = v;
  return FIB_OK;
}

int fib_set_graphs(fib_t* c, int32_t enable) {
  if (int rc = check_ctx(c)) return rc;
  c->graphs = enable != 0;
  return FIB_OK;
}

int fib_graph_replays(fib_t* c, int64_t* n) {
  if (int rc = check_ctx(c)) return rc;
  if (!n) return fail(FIB_EINVAL, "null output");
  *n = c->graph_replays;
  return FIB_OK;
}

int fib_set_kernel_timing(fib_t* c, int32_t enable) {
  if (int rc = check_ctx(c)) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  kt_harvest(c, true);
  for (int k = 0; k < FIB_KT_COUNT; ++k) {
    c->kt_ms[k] = 0.0;
    c->kt_n[k] = 0;
  }
  c->kt_on = enable != 0;
  return FIB_OK;
}

int fib_kernel_time(fib_t* c, int32_t cls, double* ms, int64_t* launches) {
  if (int rc = check_ctx(c)) return rc;
  if (cls < 0 || cls >= FIB_KT_COUNT) return fail(FIB_EINVAL, "unknown kernel class %d", cls);
  if (!ms || !launches) return fail(FIB_EINVAL, "null output");
  HIP_TRY(hipStreamSynchronize(c->stream));
  kt_harvest(c, true);
  *ms = c->kt_ms[cls];
  *launches = c->kt_n[cls];
  return FIB_OK;
}

int fib_surrogate_fallbacks(fib_t* c, int64_t* total, int64_t* steps) {
  if (int rc = check_ctx(c)) return rc;
  if (!total || !steps) return fail(FIB_EINVAL, "null output");
  *total = 0;
  *steps = 0;
  if (!c->d_sur_total) return FIB_OK;
  unsigned long long v = 0;
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(&v, c->d_sur_total, sizeof v, hipMemcpyDeviceToHost));
  *total = (int64_t)v;
  *steps = c->sur_steps;
  return FIB_OK;
}

int fib_set_adaptive(fib_t* c, double tol) {
  if (int rc = check_ctx(c)) return rc;
  if (!(std::isfinite(tol) && tol >= 0.0)) return fail(FIB_EINVAL, "tol must be finite and >= 0");
  if (tol == 0.0) {
    c->adapt_tol = 0.0;
    return FIB_OK;
  }
  if (c->sur_on)
    return fail(FIB_EUNSUPPORTED, "adaptive computation and the surrogate step do not combine");
  if (c->p.model == FIB_MODEL_ST57_APX)
    return fail(FIB_EUNSUPPORTED, "adaptive computation holds the exact models only");
  HIP_TRY(hipStreamSynchronize(c->stream));
  const size_t nt = (size_t)std::max<int64_t>(c->n_total, 1), nf = (size_t)std::max(c->n_fibers, 1);
  if (!c->d_pt) {
    std::vector<int32_t> fib_of(nt, 0);
    for (int32_t f = 0; f < c->n_fibers; ++f)
      for (int64_t i = c->offsets[f]; i < c->offsets[f + 1]; ++i) fib_of[i] = f;
    if (hipMalloc(&c->d_node_fiber, sizeof(int32_t) * nt) != hipSuccess ||
        hipMalloc(&c->d_first_on, sizeof(int32_t) * nf) != hipSuccess ||
        hipMalloc(&c->d_pt, 2 * nt) != hipSuccess || hipMalloc(&c->d_fiber_any, 2 * nf) != hipSuccess ||
        hipMalloc(&c->d_adapt_count, sizeof(unsigned long long) * fib::kAdaptCounters) != hipSuccess) {
      (void)hipFree(c->d_node_fiber);
      (void)hipFree(c->d_first_on);
      (void)hipFree(c->d_pt);
      (void)hipFree(c->d_fiber_any);
      (void)hipFree(c->d_adapt_count);
      c->d_node_fiber = c->d_first_on = nullptr;
      c->d_pt = c->d_fiber_any = nullptr;
      c->d_adapt_count = nullptr;
      return fail(FIB_ENOMEM, "device allocation failed");
    }
    HIP_TRY(hipMemcpy(c->d_node_fiber, fib_of.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice));
  }
  if (c->p.model == FIB_MODEL_ST57 && !c->d_adapt_list) {
    if (c->n_total > INT32_MAX)
      return fail(FIB_EUNSUPPORTED, "adaptive ST57 lists nodes as 32-bit indices");
    if (hipMalloc(&c->d_adapt_list, sizeof(int32_t) * nt) != hipSuccess ||
        hipMalloc(&c->d_adapt_lcount, sizeof(int32_t) * 2) != hipSuccess) {
      (void)hipFree(c->d_adapt_list);
      (void)hipFree(c->d_adapt_lcount);
      c->d_adapt_list = c->d_adapt_lcount = nullptr;
      return fail(FIB_ENOMEM, "device allocation failed");
    }
  }
  if (c->n_fibers > 0)
    HIP_TRY(hipMemcpy(c->d_first_on, c->first_on.data(), sizeof(int32_t) * c->n_fibers,
                      hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(c->d_pt, fib::PT_ACTIVE, 2 * nt));
  HIP_TRY(hipMemset(c->d_fiber_any, 0, 2 * nf));
  HIP_TRY(hipMemset(c->d_adapt_count, 0, sizeof(unsigned long long) * fib::kAdaptCounters));
  c->adapt_par = 0;
  c->adapt_tol = tol;
  return FIB_OK;
}

int fib_adaptive_solved(fib_t* c, int64_t* node_steps) {
  if (int rc = check_ctx(c)) return rc;
  if (!node_steps) return fail(FIB_EINVAL, "null argument");
  *node_steps = 0;
  if (!c->d_adapt_count) return FIB_OK;
  unsigned long long h[fib::kAdaptCounters];
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(h, c->d_adapt_count, sizeof(h), hipMemcpyDeviceToHost));
  unsigned long long sum = 0;
  for (unsigned long long v : h) sum += v;
  *node_steps = (int64_t)sum;
  return FIB_OK;
}

int fib_adaptive_points(fib_t* c, uint8_t* active, int64_t n) {
  if (int rc = check_ctx(c)) return rc;
  if (n != c->n_total || (n > 0 && !active)) return fail(FIB_EINVAL, "expected %lld values",
                                                         (long long)c->n_total);
  if (!c->d_pt) return fail(FIB_ESTATE, "adaptive computation was never enabled");
  if (n == 0) return FIB_OK;
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(active, c->d_pt + (size_t)c->adapt_par * c->n_total, (size_t)n,
                    hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n; ++i) active[i] = (active[i] & fib::PT_ACTIVE) ? 1 : 0;
  return FIB_OK;
}

int fib_get_tact(fib_t* c, float* t_act, int64_t n) {
  if (int rc = check_ctx(c)) return rc;
  if (n != c->n_total) return fail(FIB_EINVAL, "expected %lld values", (long long)c->n_total);
  if (n == 0) return FIB_OK;
  if (!t_act) return fail(FIB_EINVAL, "null output");
  HIP_TRY(hipMemcpyAsync(t_act, c->d_tact, sizeof(float) * n, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return FIB_OK;
}

int fib_reset_observables(fib_t* c) {
  if (int rc = check_ctx(c)) return rc;
  HIP_TRY(fib::launch_fill(c->d_tact, c->n_total, INFINITY, c->stream));
  return FIB_OK;
}

int fib_sync(fib_t* c) {
  if (int rc = check_ctx(c)) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  int flag = 0;
  HIP_TRY(hipMemcpy(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) return fail(FIB_ENONFINITE, "a kernel saw a non-finite membrane voltage");
  return FIB_OK;
}

}  // extern "C"
