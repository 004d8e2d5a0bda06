// Internal declarations shared by the host runtime (fib_api.hip) and the
// kernels (fib_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fib {

// Stimulus entry as the kernels see it: step indices as int32.
struct StimDev {
  int32_t on;      // first split step the entry is on in
  int32_t dur;     // consecutive split steps it stays on
  int32_t period;  // 0: single pulse
  float amp;       // current entries: uA/cm^2; voltage entries: V_m - rest_V (mV)
  int32_t voltage; // 0: current entry, 1: prescribed V_m
};

// Per-slot descriptor of the fused / diffusion kernels.
//   bit 0: the node has a left neighbour in the same fiber
//   bit 1: the node has a right neighbour in the same fiber
//   bit 2: the slot holds a real node (not padding)
//   bits 3..31: stimulus entry + 1 (0: none)
constexpr uint32_t SLOT_L = 1u;
constexpr uint32_t SLOT_R = 2u;
constexpr uint32_t SLOT_REAL = 4u;
constexpr int SLOT_STIM_SHIFT = 3;

constexpr int MAX_STATES = 64;

// FP32 in global memory.  Kernels that hide a pointer from the optimizer
// (an empty asm with the pointer as operand) type it this way: through a
// generic pointer the accesses compile to flat instructions, which also
// count against the LDS wait counter.
typedef __attribute__((address_space(1))) float gfloat;

// Point flags of the adaptive computation, one byte per node and step:
//   PT_SOLVE:  the node is solved in this step (set by the start kernel,
//              consumed by the finish kernel of a Strang step);
//   PT_ACTIVE: the last equilibrium check found the node active.
constexpr uint8_t PT_SOLVE = 1u;
constexpr uint8_t PT_ACTIVE = 2u;
// Counters of solved node-steps (spread over addresses to keep the atomics
// apart).
constexpr int kAdaptCounters = 256;
// Fibers a bin may hold for the fused kernel with adaptive computation.
constexpr int kBinFibers = 64;

// Everything a kernel launch needs, passed by value.
struct KArgs {
  float* state;             // SoA [S][n_total]
  int64_t n_total;
  const int32_t* slot_gidx; // [groups * cap], -1 for padding
  const uint32_t* slot_info;// [groups * cap]
  const int32_t* node_stim; // [n_total], stimulus entry + 1 (0: none)
  const StimDev* stim;      // stimulus table
  float* t_act;             // [n_total]
  float* v_prev;            // [n_total], V_m at the end of the previous split step (SPLIT)
  float* samples;           // [rows][n_total] or null
  int64_t sample_every;     // 0: no samples
  int64_t sample_row0;      // rows written by earlier calls: step0 / sample_every
  int64_t sample_rows;      // capacity of `samples`
  int* flag;                // bit 0: non-finite V_m seen
  int32_t cap;              // slots per group = threads * nodes_per_thread
  int32_t step0;
  int32_t n_steps;
  int32_t n_sub;            // reaction substeps before the diffusion (Strang: half a
                            // split step; Godunov: the whole step) and per k_react phase
  int32_t n_sub2;           // fused kernel: reaction substeps after the diffusion
                            // (Strang: n_sub; Godunov: 0)
  int32_t n_cn;             // diffusion substeps per split step
  int32_t pcr_levels;       // reduced-system PCR levels
  float dt;                 // split step (ms)
  float tau;                // reaction substep (ms)
  float r_mat;              // 2 theta c dt_cn / h^2 with c = sigma / (Am Cm): the row
                            // weights of the matrix I - theta dt_cn L
  float rhs;                // 1 / theta: dt_cn L V from the matrix's row weights
  float inv_cm;             // 1 / Cm
  float v_th;               // activation threshold (mV)
  // adaptive computation (split schedule; all null when off)
  const int32_t* node_fiber;      // [n_total] fiber of each node
  const int32_t* fiber_first_on;  // [n_fibers] first split step with a stimulus entry on
  const uint8_t* pt_prev;         // [n_total] point flags after the previous step
  uint8_t* pt_cur;                // [n_total] point flags of this step
  uint8_t* fiber_any;             // [n_fibers] 1: a node of the fiber is solved in this step
  uint8_t* fiber_any_next;        // [n_fibers] flags of the next step (cleared by the diffusion)
  unsigned long long* adapt_count;// [kAdaptCounters] solved node-steps
  float adapt_tol;                // relative change of an active point
  const uint8_t* slot_fiber;      // fused: [groups * cap] bin-local fiber of each slot
  const int32_t* bin_first_on;    // fused: [groups * kBinFibers] first stimulus step
  // graph replays of the split schedule: a device value added to the step
  // arguments of the reaction, surrogate and fallback kernels (null: none)
  const int32_t* step_base;
  // fibers of each bin for the split-schedule diffusion: entries
  // bin_ent[b] .. bin_ent[b + 1] - 1 list bin b's fibers in slot order and
  // end with an entry whose start is the bin's load
  const int32_t* bin_ent;   // [groups + 1]
  const int32_t* ent_s0;    // first slot of the entry's fiber in its bin
  const int32_t* ent_gofs;  // first node of the entry's fiber
  const int32_t* ent_fiber; // the entry's fiber
  int32_t max_ents;         // the most entries of one bin (end entry included)
  int32_t n_bins;           // bins (workgroups of the fused kernels)
  float rest[MAX_STATES];   // resting state (FP32); device rows hold y_k - rest[k]
};

// Whether entry e is on during split step n: a pulse of `dur` steps from
// `on`, repeated every `period` steps if > 0.
__device__ __forceinline__ bool stim_on(const StimDev& e, int32_t n) {
  int32_t k = n - e.on;
  if (k < 0) return false;
  if (e.period > 0) k = k % e.period;
  return k < e.dur;
}

// Whether stimulus entry `sid1 - 1` (0: none), of either kind, is on during
// split step n.
__device__ __forceinline__ bool stim_any_on(uint32_t sid1, const StimDev* __restrict__ tab,
                                            int32_t n) {
  return sid1 != 0 && stim_on(tab[sid1 - 1], n);
}

// Current of stimulus entry `sid1 - 1` (0: none) during split step n
// (0 for voltage entries).
__device__ __forceinline__ float stim_current(uint32_t sid1, const StimDev* __restrict__ tab,
                                              int32_t n) {
  if (sid1 == 0) return 0.0f;
  const StimDev e = tab[sid1 - 1];
  return (!e.voltage && stim_on(e, n)) ? e.amp : 0.0f;
}

// Current of entry `sid1 - 1` during split step n, and the prescription of
// a voltage entry: returns true with v_off = V_m - rest_V if the node's V_m
// is set at the start of step n.
__device__ __forceinline__ bool stim_eval(uint32_t sid1, const StimDev* __restrict__ tab,
                                          int32_t n, float& I, float& v_off) {
  I = 0.0f;
  if (sid1 == 0) return false;
  const StimDev e = tab[sid1 - 1];
  if (!stim_on(e, n)) return false;
  if (!e.voltage) {
    I = e.amp;
    return false;
  }
  v_off = e.amp;
  return true;
}

// Read-only view of a context for the EMG module (emg.hip).
struct CtxView {
  int32_t n_fibers;
  const int32_t* n_nodes;  // host, n_fibers entries
  int64_t n_total;
  float* d_state;          // device state; row 0 holds V_m - rest_V
  double h;                // node spacing along the fibers (cm)
  hipStream_t stream;
  bool state_ready;
  int model;
};
}  // namespace fib
struct fib_ctx;
namespace fib {
CtxView ctx_view(const fib_ctx* c);
int set_error(int code, const char* msg);

// Launchers (fib_kernels.hip).  Each returns the hipError_t of the launch.
// Largest workgroup size the kernels are built for with K nodes per thread
// (0: K not supported).
int plan_max_threads(int K);
hipError_t launch_run_fused(int model, int K, int groups, int threads, size_t lds_bytes,
                            const KArgs& a, hipStream_t s);
// Fused kernel with adaptive computation (Hodgkin-Huxley); lds_bytes =
// lds_bytes_for(threads, levels) + adapt_lds_extra(cap).
hipError_t launch_run_fused_adaptive(int K, int groups, int threads, size_t lds_bytes,
                                     const KArgs& a, hipStream_t s);
hipError_t launch_diffusion(int K, int groups, int threads, size_t lds_bytes, const KArgs& a,
                            hipStream_t s);
// Reaction kernel with states in device memory; flags: 1 = reaction with the
// stimulus current of step_a, 2 = observables after step_a, 4 = the start of
// step_b: its V_m prescriptions, then reaction with its current (applied in
// that order).
hipError_t launch_react(int model, int32_t step_a, int32_t step_b, int flags, const KArgs& a,
                        hipStream_t s);
// Adaptive computation, split schedule.  Start of split step `step`: the
// observables of step - 1 if observe_prev, the points to solve (from the
// flags of the previous step and the stimulus), their V_m prescriptions and
// the reaction part before the diffusion; with Godunov splitting (the
// step's only reaction part) also their equilibrium check.  Hodgkin-Huxley
// models only (ST57 takes the list form below).
hipError_t launch_adapt_start(int model, bool godunov, int32_t step, bool observe_prev,
                              const KArgs& a, hipStream_t s);
// End of Strang split step `step`: the second reaction half and the
// equilibrium check of the solved points, then the observables
// (Hodgkin-Huxley models).
hipError_t launch_adapt_finish(int model, int32_t step, const KArgs& a, hipStream_t s);
// The adaptive split steps for ST57: decisions and a list of the solved
// nodes (counts[slot]; counts[slot ^ 1] is cleared), the reaction parts over
// that list (phase 0: Strang start, 1: Strang end, 2: Godunov step), and the
// observables of every node (after a run's last step).
hipError_t launch_adapt_decide(bool godunov, int32_t step, bool observe_prev, int* list,
                              int* counts, int slot, const KArgs& a, hipStream_t s);
hipError_t launch_adapt_solve(int model, int phase, int32_t step, const int* list,
                              const int* count, const KArgs& a, hipStream_t s);
hipError_t launch_observe(int32_t step, const KArgs& a, hipStream_t s);
hipError_t launch_init(int model, const float* vm_noise, const float* rel_noise, const KArgs& a,
                       hipStream_t s);
hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s);
// Node-major copies for training data: U[i][k] = state[k][i]; state[k][i] =
// U[r0 + i][k] (0 past n); dU[r0 + i][k] = state[k][i] - U[r0 + i][k].
hipError_t launch_state_rows(const float* state, int64_t nt, int S, float* U, hipStream_t s);
hipError_t launch_rows_to_state(const float* U, int64_t r0, int64_t n, int S, float* state,
                                int64_t nt, hipStream_t s);
hipError_t launch_state_minus_rows(const float* state, const float* U, int64_t r0, int64_t n, int S,
                                   int64_t nt, float* dU, hipStream_t s);
// *p = v (set) or *p += v, by one thread: the step base of graph replays.
hipError_t launch_step_base(int32_t* p, int32_t v, bool set, hipStream_t s);

// The device step base as a kernel sees it: 0 without graph replay.
__device__ __forceinline__ int32_t step_base_of(const KArgs& a) {
  return a.step_base ? *a.step_base : 0;
}
hipError_t launch_check_finite(const float* p, int64_t n, int* flag, hipStream_t s);

// LDS bytes the fused / diffusion kernels need for `threads` threads and
// `levels` PCR levels.
inline size_t lds_bytes_for(int threads, int levels) {
  return sizeof(float) * (size_t)threads * (size_t)(6 + 2 * levels);
}

// LDS of the split-schedule diffusion: the staged V of every slot (cap
// floats) and its coupling bits (cap bytes), then the solve's arrays (the
// separate setup and solve's 6 + 2L floats per thread, or the merged
// single-substep solve's 12), then two buffers of bin entries (starts,
// first nodes, fibers: 3 max_ents ints each).
__host__ __device__ inline size_t diffusion_stage_part(int cap) {
  return (5 * (size_t)cap + 15) & ~(size_t)15;
}
__host__ __device__ inline size_t diffusion_region_bytes(int threads, int levels, int cap) {
  const size_t per = (size_t)(6 + 2 * levels) > 12 ? (size_t)(6 + 2 * levels) : 12;
  return diffusion_stage_part(cap) + sizeof(float) * (size_t)threads * per;
}
inline size_t diffusion_lds_bytes(int threads, int levels, int cap, int max_ents) {
  return diffusion_region_bytes(threads, levels, cap) + 24 * (size_t)max_ents;
}

// LDS the adaptive fused kernel needs beyond the Crank-Nicolson region for
// a bin of `cap` slots (a multiple of 64): the states (4 cap floats), the
// compacted list of solved slots (cap uint16), the bin-local fiber of each
// slot (cap bytes), the verdict bits (cap / 32 + 2 words), the per-fiber
// flags of two steps, and two list lengths and two flags.
inline size_t adapt_lds_extra(int cap) {
  return (size_t)cap * (16 + 2 + 1) + 4 * ((size_t)cap / 32 + 2) + 2 * kBinFibers + 4 * 4;
}

}  // namespace fib
