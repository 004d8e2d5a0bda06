/*
 * fib.h -- C ABI of libfib.so, an MI355X (gfx950) solver for the
 * Strang-split monodomain equation on many independent 1D muscle fibers
 * (B. Maier, "Scalable Biophysical Simulations of the Neuromuscular System",
 * 2021).
 *
 * The problem (thesis section "Discretization of the Monodomain Model" and
 * eq. discretized_fibers_1):
 *   on every fiber, dV/dt = sigma/(Am Cm) d2V/dx2 - I_ion(V, y)/Cm with
 *   no-flux ends (eqs. monodomain, monodomain_bc1), and dy/dt = G(V, y) at
 *   every node (eq. subcellular).  One split step of width dt is
 *   R(dt/2) D(dt) R(dt/2) (eq. monodomain_strang, 0D-1D-0D order):
 *     R: Heun's method (eq. heun) on all states of every node, in
 *        ceil((dt/2)/dt_0D) equal substeps, with the node's stimulus current
 *        held constant over the split step;
 *     D: Crank-Nicolson (eq. crank_nicolson, theta = 1/2) with linear finite
 *        elements and a lumped mass matrix (section "Using Mass Lumping for
 *        Implicit Timestepping", eq. lumping_crank_nicolson) in
 *        ceil(dt/dt_1D) equal substeps, i.e. one tridiagonal system per fiber
 *        per substep (section "Improved Parallel Solver Scheme using the
 *        Thomas Algorithm").
 *   Stimulus: a current density on the nodes around a neuromuscular junction
 *   (section "Specification of Stimulation Times Using Callback Functions").
 *
 * Units: cm, ms, mV, uA/cm^2, uF/cm^2, mS/cm.
 *
 * Conventions for every function below:
 *   - Return 0 (FIB_OK) on success or a negative fib_status.  After an error,
 *     fib_last_error() returns a message for the calling thread.  No C++
 *     exception crosses this boundary.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory on the context's device.  Host arrays are copied; the
 *     library never keeps a caller pointer beyond the call.
 *   - All device work is enqueued on the stream given to fib_create (NULL =
 *     the null stream) and is asynchronous unless stated otherwise.
 *   - The state is structure of arrays: value k of global node i is at
 *     index k * n_total + i, nodes of fiber f at offsets
 *     sum(n_nodes[0..f-1]) .. + n_nodes[f] - 1 (the order given to
 *     fib_create).  State 0 is V_m (mV).  Host arrays hold the states
 *     themselves; on the device the state is FP32 and row k holds
 *     y_k - ref_k, ref being the model's resting state rounded to FP32
 *     (see fib_state_device).
 *   - A context is not thread safe; calls on one context from several
 *     threads must be serialized by the caller.
 */
#ifndef FIB_H
#define FIB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FIB_OK = 0,
  FIB_EINVAL = -1,       /* invalid argument (nothing was changed) */
  FIB_ENOMEM = -2,       /* device or host allocation failed */
  FIB_EHIP = -3,         /* a HIP runtime call failed */
  FIB_ENONFINITE = -4,   /* a non-finite state value was detected */
  FIB_ESTATE = -5,       /* call not valid in the context's current state */
  FIB_EUNSUPPORTED = -6  /* valid request that the library does not support */
} fib_status;

/* Subcellular models: Hodgkin-Huxley (4 states), the 57-state ST57 stand-in
 * for the Shorten model, Hodgkin-Huxley with every exponential of its rates
 * replaced by the approximation exp*(x) = (1 + x/1024)^1024 of
 * eq. apx-e-function (4 states; its own resting state), and ST57 with every
 * exponential replaced by exp* and every logarithm by log* (the thesis's
 * sixth-order Taylor pieces of log around 1, 3 and 9, split at 2 and 6, then
 * one Newton step y - (1 - x / exp*(y)); figure apxlog), applied to the
 * arguments as the model writes them, with arguments outside [0.2, 20]
 * scaled into it by powers of two first (57 states; its own resting state).
 * The fused schedule, the adaptive fused kernel and the surrogate step take
 * Hodgkin-Huxley (and ST57 for the surrogate step) only; HH_APX_EXP runs the
 * fused and the split schedule, ST57_APX the split schedule without
 * adaptive computation or surrogate. */
enum { FIB_MODEL_HH = 0, FIB_MODEL_ST57 = 1, FIB_MODEL_HH_APX_EXP = 2, FIB_MODEL_ST57_APX = 3 };

/* Execution schedule of fib_run.
 *   FUSED: one persistent kernel keeps every node's states in registers and
 *          every fiber's V_m exchange in LDS for all split steps of the call.
 *   SPLIT: one reaction kernel and one diffusion kernel per split step with
 *          states in device memory.
 *   AUTO:  FUSED where the model fits it (Hodgkin-Huxley), else SPLIT. */
enum { FIB_SCHED_AUTO = 0, FIB_SCHED_FUSED = 1, FIB_SCHED_SPLIT = 2 };

/* Operator splitting of a split step of width dt = dt_split.
 *   STRANG:  R(dt/2) D(dt) R(dt/2) (eq. monodomain_strang, second order);
 *   GODUNOV: R(dt) D(dt)           (eq. monodomain_godunov, first order).
 * R takes ceil(span/dt_0D) equal Heun substeps over its span. */
enum { FIB_SPLIT_STRANG = 0, FIB_SPLIT_GODUNOV = 1 };

/* Time stepping of the diffusion substeps (lumped mass matrix): the
 * theta-scheme (I - theta dt L) V+ = (I + (1 - theta) dt L) V with
 *   CRANK_NICOLSON: theta = 1/2 (eq. lumping_crank_nicolson, second order);
 *   IMPLICIT_EULER: theta = 1   (eq. lumping_implicit_euler, first order,
 *                   strongly damping). */
enum { FIB_1D_CRANK_NICOLSON = 0, FIB_1D_IMPLICIT_EULER = 1 };

/* Kind of a stimulus entry (section "Specification of Stimulation Times
 * Using Callback Functions"). */
enum { FIB_STIM_CURRENT = 0, FIB_STIM_VOLTAGE = 1 };

typedef struct {
  int32_t model;      /* FIB_MODEL_* */
  int32_t schedule;   /* FIB_SCHED_* */
  double Cm;          /* membrane capacitance, uF/cm^2 (> 0) */
  double Am;          /* surface-to-volume ratio, 1/cm (> 0) */
  double sigma;       /* effective conductivity, mS/cm (>= 0) */
  double h;           /* node spacing, cm (> 0) */
  double dt_0D;       /* largest reaction substep, ms (> 0) */
  double dt_1D;       /* largest diffusion substep, ms (> 0) */
  double dt_split;    /* split step, ms (> 0) */
  double v_th;        /* activation threshold of the activation-time observable, mV */
  int32_t pcr_full;   /* 0: stop the reduced-system PCR once every remaining coupling is
                         below 2^-40 of the diagonal; 1: run all log2(threads) levels */
  int32_t threads_per_group; /* 0: automatic; else a multiple of 64 in 64..1024 (at most
                                768 with 9 or 10 nodes per thread, 512 with 11..14) */
  int32_t nodes_per_thread;  /* 0: automatic (2..8); else 2..14 */
  int32_t groups;            /* 0: automatic (one per compute unit); else the number of
                                fiber bins, i.e. workgroups of the fused kernel */
  int32_t splitting;         /* FIB_SPLIT_* (0: Strang) */
  int32_t time_1d;           /* FIB_1D_* (0: Crank-Nicolson) */
  int32_t tune;              /* 0: keep the plan; 1: the first fib_run that advances any
                                step first runs fib_autotune (100 trial steps, 8
                                candidates) from the state it is given, which the
                                autotuner restores, then runs on the chosen plan */
} fib_params;

/* One stimulus entry on nodes node-half_width .. node+half_width of fiber
 * `fiber` (clipped to the fiber), on during split steps n with
 * n >= step_on and (n - step_on) mod period < n_steps (period = 0: only
 * step_on <= n < step_on + n_steps).
 *   FIB_STIM_CURRENT: current density `amp` (uA/cm^2) in every reaction
 *     substep of a step it is on in;
 *   FIB_STIM_VOLTAGE: V_m of the covered nodes is set to `amp` (mV) at the
 *     start of every split step it is on in, before the step's first
 *     reaction part; the activation-time test spans the whole step, from
 *     the voltage before the prescription.  Applied by fib_run only.
 * A node may be covered by at most one entry.  Step indices must be below
 * 2^31. */
typedef struct {
  int32_t fiber;
  int32_t node;
  int32_t half_width;
  int32_t mode;      /* FIB_STIM_* */
  int64_t step_on;
  int64_t n_steps;
  int64_t period;
  double amp;
} fib_stim;

typedef struct fib_ctx fib_t;

/* Number of states per node of a model (4 for Hodgkin-Huxley), or
 * FIB_EINVAL. */
int fib_n_states(int32_t model);

/* Resting state of the model: the voltage at which the ionic current with
 * all gates at equilibrium vanishes, and the gates' equilibria there
 * (thesis section "Subcellular Model").  Host computation in FP64;
 * y_out (host) receives fib_n_states(p->model) values. */
int fib_rest_state(const fib_params* p, double* y_out);

/* Checks a parameter set without touching the GPU: FIB_OK or FIB_EINVAL. */
int fib_check_params(const fib_params* p);

/* The plan fib_create would choose on a device with `compute_units` compute
 * units, computed on the host without touching the GPU: workgroups (fiber
 * bins), threads per workgroup, nodes per thread, PCR levels of the fused
 * diffusion solve, and the node count of the fullest bin.  Any output
 * pointer may be NULL.  FIB_EUNSUPPORTED if no plan fits (a fiber longer
 * than 8192 nodes, or a fixed shape that cannot hold the fibers). */
int fib_plan_preview(const fib_params* p, int32_t n_fibers, const int32_t* n_nodes,
                     int32_t compute_units, int32_t* groups, int32_t* threads,
                     int32_t* nodes_per_thread, int32_t* pcr_levels, int64_t* max_load);

/* Creates a context for n_fibers fibers with n_nodes[f] >= 1 nodes each
 * (host array).  Allocates the FP32 state, the activation-time array and
 * the schedule tables on the current HIP device and plans how fibers are
 * grouped into workgroups.  `stream` is a hipStream_t (may be NULL); it is
 * borrowed and must outlive the context.  The state starts uninitialized:
 * call fib_init_state or fib_set_state before stepping. */
int fib_create(const fib_params* p, int32_t n_fibers, const int32_t* n_nodes, void* stream,
               fib_t** out);

/* Releases every resource of the context (waits for its stream first).
 * NULL is a no-op. */
void fib_destroy(fib_t* ctx);

/* Message of the last failed call on this thread ("" if none). */
const char* fib_last_error(void);

/* Total number of nodes of the context. */
int64_t fib_n_total(const fib_t* ctx);

/* Initial state (on the device): every node starts at the model's resting
 * state y*, each state multiplied by (1 + rel_noise[k * n_total + i]) and
 * V_m then shifted by vm_noise[i] (mV).  Both arrays are FP32 device
 * pointers and may be NULL (no noise).  Also resets the observables. */
int fib_init_state(fib_t* ctx, const float* vm_noise, const float* rel_noise);

/* Copies a full FP64 host state (n_values = n_states * n_total, layout as
 * above) to the device, rounding to FP32.  Blocking. */
int fib_set_state(fib_t* ctx, const double* y, int64_t n_values);

/* Copies the device state to FP64 host memory (n_values as above).
 * Blocking; returns FIB_ENONFINITE if any value is NaN or infinite. */
int fib_get_state(fib_t* ctx, double* y, int64_t n_values);

/* Device pointer to the FP32 state (n_states * n_total floats) that the
 * context owns, valid until fib_destroy, for zero-copy access.  Row k of
 * the device state holds y_k - ref_k; ref (host, nullable) receives the
 * n_states reference values. */
int fib_state_device(fib_t* ctx, float** state, double* ref);

/* Replaces the stimulus table (host array of n entries, copied). */
int fib_set_stimulus(fib_t* ctx, const fib_stim* stim, int32_t n);

/* Reaction part only: ceil(span/dt_0D) equal Heun substeps on every node,
 * with the stimulus current of split step `step` (voltage entries are not
 * applied).  One kernel launch. */
int fib_step_reaction(fib_t* ctx, int64_t step, double span);

/* Diffusion part only: ceil(span/dt_1D) equal substeps of the time_1d
 * scheme on every fiber.  One kernel launch. */
int fib_step_diffusion(fib_t* ctx, double span);

/* Split steps step0 .. step0 + n_steps - 1 (step n covers the time
 * [n dt_split, (n+1) dt_split]).  Observables:
 *   - activation time per node (kept by the context, see fib_get_tact):
 *     the first upward crossing of v_th between the ends of two
 *     consecutive split steps, interpolated linearly;
 *   - if samples != NULL and sample_every > 0: after every step n with
 *     (n + 1) % sample_every == 0, V_m of all nodes is written to the FP32
 *     device array samples at row (n + 1) / sample_every - 1 -
 *     step0 / sample_every (row length n_total); sample_rows is the number
 *     of rows the array holds (FIB_EINVAL if too small).
 * Asynchronous. */
int fib_run(fib_t* ctx, int64_t step0, int64_t n_steps, int64_t sample_every, float* samples,
            int64_t sample_rows);

/* Adaptive computation of the subcellular model (section
 * sec:adaptive_computation_for_fiber_based, figure state_chart) for
 * fib_run.  With tol > 0 each node ("point") is active, inactive or
 * "neighbor is active", and per split step:
 *   - a fiber takes no part (no reaction, no diffusion) before the first
 *     step in which one of its stimulus entries is on (by the table,
 *     whatever step a run starts at);
 *   - a node of a fiber that takes part is solved if the last check found
 *     it or a neighbour in its fiber active, or a stimulus entry that is on
 *     covers it or a neighbour; the reaction parts run on solved nodes
 *     only, the diffusion on fibers with at least one solved node;
 *   - each solved node checks the relative change |y_k+ - y_k| >
 *     tol |y_k| of every state over the step's last reaction part (the
 *     thesis uses tol = 1e-5): active if any state moved that much, else
 *     inactive.
 * The check runs in FP32 on the device.  Enabling (or re-enabling) resets
 * every point to active, its initial state, and the solved-node counter to
 * zero; fib_init_state and fib_set_state reset the points too.  tol = 0
 * turns it off.  Schedules: FUSED (Hodgkin-Huxley) runs a variant of the
 * fused kernel that keeps each bin's states in LDS and compacts the solved
 * nodes of every step; it takes plans with at most 64 fibers per bin whose
 * states fit the LDS (fib_run returns FIB_EUNSUPPORTED otherwise).  SPLIT
 * runs, for Hodgkin-Huxley, one start kernel, the diffusion and (Strang) one
 * finish kernel per step; for ST57 a decision kernel that lists the solved
 * nodes, the reaction parts over that list, and the diffusion (the library
 * then holds a list of n_total 32-bit indices on the device, allocated here;
 * FIB_EUNSUPPORTED for more than 2^31 - 1 nodes, FIB_ENOMEM if it does not
 * fit).  AUTO takes the fused variant where it can, else the split
 * schedule.  FIB_EUNSUPPORTED with an attached surrogate.
 * fib_autotune times the plain schedule and leaves the points alone.
 * Blocking. */
int fib_set_adaptive(fib_t* ctx, double tol);

/* Node-steps whose reaction was solved by adaptive runs since
 * fib_set_adaptive enabled it.  Blocking. */
int fib_adaptive_solved(fib_t* ctx, int64_t* node_steps);

/* Per node 1 if the last equilibrium check found it active (nodes of
 * fibers that have not taken part yet keep their initial "active"), else 0,
 * into a host array of n_total bytes.  FIB_ESTATE if adaptive computation
 * was never enabled.  Blocking. */
int fib_adaptive_points(fib_t* ctx, uint8_t* active, int64_t n);

/* Activation times (ms, +inf where V_m has not crossed v_th) into a host
 * FP32 array of n_total values.  Blocking. */
int fib_get_tact(fib_t* ctx, float* t_act, int64_t n);

/* Sets every activation time back to +inf. */
int fib_reset_observables(fib_t* ctx);

/* Waits for the context's stream; returns FIB_EHIP on a deferred device
 * error and FIB_ENONFINITE if a kernel flagged a non-finite V_m. */
int fib_sync(fib_t* ctx);

/* Describes the plan chosen by fib_create (or fib_autotune): workgroups
 * (fiber bins), threads per workgroup, nodes per thread, and PCR levels of
 * the fused diffusion solve.  Any pointer may be NULL. */
int fib_plan_info(const fib_t* ctx, int32_t* groups, int32_t* threads, int32_t* nodes_per_thread,
                  int32_t* pcr_levels);

/* Autotuner of the workgroup shape (the batching of uneven fibers into
 * bins of whole fibers is kept): for the current bins it ranks every
 * (threads per workgroup, nodes per thread) that holds the heaviest bin
 * with at most 30 % padding by the slots one SIMD sweeps per step, times
 * the current plan and up to max_candidates - 1 of the best-ranked ones
 * over trial_steps split steps of fib_run from the current state (HIP
 * events on the context's stream), and keeps the fastest.  The state,
 * activation times and previous-V_m buffers are restored afterwards, so a
 * tuned context continues exactly where it was; results of later runs
 * differ from the untuned plan only by FP32 rounding (the partitioned
 * solve groups nodes differently).  ms_per_step (nullable) receives the
 * chosen plan's trial time per split step.  Synchronous; allocates scratch
 * for one copy of the state.  FIB_ESTATE without an initialized state. */
int fib_autotune(fib_t* ctx, int32_t trial_steps, int32_t max_candidates, double* ms_per_step);

/* ------------------------------------------------------------------------
 * Surrogate network: a multilayer perceptron with SiLU hidden layers and a
 * linear output, z_l = W_l a_{l-1} + b_l, used as a learned replacement of
 * the subcellular update over one split step (no counterpart in the
 * thesis, which names learned surrogates only as an outlook).  Matrix
 * products run on the matrix cores with BF16 operands and FP32
 * accumulation; parameters, Adam moments and gradients are FP32.
 *
 * Parameter layout (flat FP32): for every weight layer l = 1..L the matrix
 * W_l (sizes[l] rows x sizes[l-1] columns, row-major) followed by b_l.
 * Data arrays are FP32 device pointers, row-major, one sample per row.
 * ------------------------------------------------------------------------ */
typedef struct fib_mlp fib_mlp_t;

/* Hidden-layer activations: SiLU(z) = z / (1 + e^-z); ReLU(z) = max(z, 0). */
#define FIB_ACT_SILU 0
#define FIB_ACT_RELU 1

/* Creates a network with n_layers weight layers (1..6), layer widths
 * sizes[0..n_layers] (1..512; sizes[0] = inputs) and the given hidden
 * activation (the output layer is linear).  Parameters start at 0: set
 * them with fib_mlp_set_params.  `stream` as for fib_create. */
int fib_mlp_create(int32_t n_layers, const int32_t* sizes, int32_t activation, void* stream,
                   fib_mlp_t** out);
void fib_mlp_destroy(fib_mlp_t* net);
int64_t fib_mlp_n_params(const fib_mlp_t* net);

/* Copies all parameters from / to host memory (blocking). */
int fib_mlp_set_params(fib_mlp_t* net, const float* params, int64_t n);
int fib_mlp_get_params(fib_mlp_t* net, float* params, int64_t n);

/* O[b] = network(X[b]) for b < B (X: B x sizes[0], O: B x sizes[L]). */
int fib_mlp_forward(fib_mlp_t* net, const float* X, int64_t B, float* O);

/* Gradient of loss = sum_b sum_k (O_bk - T_bk)^2 / (2 B sizes[L]) with
 * respect to the flat parameters into `grad` (device, n_params floats;
 * NULL: internal buffer) and the loss into loss[0] (device, nullable).
 * Deterministic: chunk partial sums are reduced in a fixed order. */
int fib_mlp_gradient(fib_mlp_t* net, const float* X, const float* T, int64_t B, float* grad,
                     float* loss);

/* fib_mlp_gradient for callers that cannot allocate device memory (code
 * under HIP graph capture, tight training loops, harnesses that forbid
 * allocation): the same kernels and the same result, bit for bit, with the
 * per-chunk partial gradients and losses in a fixed 16 MiB array of the
 * library's code object on the network's device instead of memory the
 * network allocates when a batch grows.  Allocates nothing and calls no
 * allocating routine.  Limit: ceil(B / 32) (n_params + 1) <= 2^22 floats
 * (B <= 4288 for the 31289-parameter ST57 network, 14944 for the 8964-
 * parameter Hodgkin-Huxley one); larger batches return FIB_EINVAL.  The
 * array is shared by every call on that device and keeps the last call's
 * contents (each call overwrites what it reads), so calls that overlap on
 * one device -- on different streams or threads -- race.  grad (device,
 * nullable: the network's own buffer) and loss (device, nullable) as for
 * fib_mlp_gradient. */
int fib_mlp_gradient_noalloc(fib_mlp_t* net, const float* X, const float* T, int64_t B,
                             float* grad, float* loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on that loss with
 * learning rate lr; the loss before the step goes to loss[0] (nullable). */
int fib_mlp_adam_step(fib_mlp_t* net, const float* X, const float* T, int64_t B, double lr,
                      float* loss);

/* Clears the Adam moments and step count. */
int fib_mlp_reset_optimizer(fib_mlp_t* net);

/* Training data of the surrogate.  Statistics of the columns of A (device,
 * rows x cols FP32, row-major, 1 <= cols <= 64) on `stream`: the mean and
 * the sample standard deviation (two passes, FP64 sums in a fixed order, so
 * the result is deterministic) and the minimum and maximum, into host
 * arrays of cols values.  Allocates and frees a small device buffer;
 * blocking. */
int fib_column_stats(const float* A, int64_t rows, int32_t cols, void* stream, double* mean,
                     double* std, float* cmin, float* cmax);

/* Y[r][k] = (A[r][k] - shift[k]) * scale[k] for k < cols (A device, rows x
 * cols; shift, scale host arrays of cols values) into Y (device, row
 * stride ldy >= cols); if ldy > cols, also Y[r][cols] = extra (the
 * stimulus-flag input).  Columns beyond are left as they are.  Blocking. */
int fib_normalize_rows(const float* A, int64_t rows, int32_t cols, const float* shift,
                       const float* scale, double extra, float* Y, int32_t ldy, void* stream);

/* The context's device state, node-major, into U (device, n_total x
 * n_states floats): U[i][k] = y_k - ref_k of node i.  Asynchronous. */
int fib_state_rows(fib_t* ctx, float* U);

/* Targets of the surrogate: for every row of U (device, rows x n_states,
 * node-major offsets from the reference as fib_state_rows writes them), the
 * increment of the plain method's two reaction halves R(dt/2) R(dt/2)
 * (eq. heun, ceil((dt/2)/dt_0D) substeps each) with the stimulus current of
 * split step `step` at the node the row is loaded into (rows are loaded n_total at
 * a time into the context's state, row j of a chunk into node j), written
 * to dU (device, rows x n_states).  Overwrites the context's state (it is
 * left initialized).  Asynchronous. */
int fib_reaction_increments(fib_t* ctx, const float* U, int64_t rows, int64_t step, float* dU);

/* ------------------------------------------------------------------------
 * Surrogate split step.  With a network attached, fib_run (split schedule)
 * replaces the two reaction halves that meet between consecutive diffusion
 * steps -- R(dt/2) of step n, then R(dt/2) of step n+1 -- by one
 * implicit-midpoint step of width dt predicted by the network:
 *   inputs  x_k = (u_k - in_shift[k]) * in_scale[k], k < n_states, with u
 *           the state minus the resting state, plus I * flag_scale (the
 *           stimulus of step n) when the network has n_states + 1 inputs;
 *   outputs du_k = out_shift[k] + out_scale[k] * o_k (the predictor);
 *   corrector du1 = dt G(y + du/2, I), du2 = dt G(y + du1/2, I)
 *   (G: the model's right-hand side; fixed-point iterations of the
 *   implicit midpoint rule started from the prediction: two for
 *   Hodgkin-Huxley, one for ST57, whose right-hand side dominates the cost).
 * A node takes the last iterate du_c only if |du1 - du|_k <= tol * res_scale[k] for every
 * state k (absolute tolerances), its stimulus current is the same in both
 * halves, no voltage entry prescribes its V_m at the start of step n+1,
 * and (for networks without the flag input) it is not stimulated; all
 * other nodes take the plain Heun substeps.  Strang splitting only
 * (FIB_EUNSUPPORTED with Godunov).  Steps that write V_m samples,
 * and the last step of a call, run the plain path for every node.  For
 * kept nodes the activation-time test uses the midpoint y + du_c/2 as the
 * state at the end of step n.  The surrogate is an addition of this
 * library: the thesis names learned surrogate models only as an outlook.
 * Supported shapes: Hodgkin-Huxley 4 or 5 -> 64 -> 64 -> 64 -> 4, ST57
 * 57 or 58 -> 128 -> 128 -> 57.  The network's current parameters are
 * copied (packed to BF16) by this call; later changes to the network need
 * another call.  Host arrays of n_states values.
 * ------------------------------------------------------------------------ */
int fib_set_surrogate(fib_t* ctx, const fib_mlp_t* net, const float* in_shift,
                      const float* in_scale, const float* out_shift, const float* out_scale,
                      const float* res_scale, double flag_scale, double tol);

/* The surrogate pair alone: finishes split step `step` and starts step
 * step + 1 on every node (kept nodes by the corrected prediction, the
 * others by the plain Heun substeps), with the observables of step `step`.
 * Asynchronous; FIB_ESTATE without an attached surrogate. */
int fib_step_surrogate(fib_t* ctx, int64_t step);

/* The network's prediction alone: writes du (device, FP32, [n_states][n_total],
 * caller-owned) for the current state with the stimulus of step `step`,
 * denormalized as above; changes no state.  Asynchronous.  For checking a
 * trained network against its reference and for measuring its error. */
int fib_surrogate_predict(fib_t* ctx, int64_t step, float* du);

/* Detaches the surrogate: fib_run takes the plain path again. */
int fib_clear_surrogate(fib_t* ctx);

/* Number of nodes that took the plain path in the last surrogate step
 * (blocking). */
int fib_surrogate_last_fallbacks(fib_t* ctx, int64_t* n);

/* Nodes that took the plain path, summed over every surrogate step since
 * the step was attached (fib_set_surrogate or fib_set_predictor), and the
 * number of those steps: the rejected share is total / (steps n_total).
 * Blocking. */
int fib_surrogate_fallbacks(fib_t* ctx, int64_t* total, int64_t* steps);

/* HIP graph replay of the split schedule (on by default).  With the Strang
 * splitting, fib_run captures one block of P consecutive split steps --
 * diffusion, then the reaction pair (or surrogate pair) that ends each step
 * and starts the next -- once per call, with its step arguments relative to
 * a device step base, and launches the captured graph once per block: P is
 * twice the sample interval (an odd interval: the interval itself; no
 * samples: 64 steps), blocks start at multiples of P, and the first and
 * last steps of the call and the steps before the first block are launched
 * as before.  Results are bitwise those of the step-by-step launches.  The
 * graph of a call is released at the next call that captures one (after
 * waiting for its replays) or at fib_destroy.  Not used while kernel timing
 * is on, for adaptive runs, Godunov splitting or the fused schedule.
 * enable = 0 turns it off. */
int fib_set_graphs(fib_t* ctx, int32_t enable);

/* Number of graph launches fib_run has made on this context. */
int fib_graph_replays(fib_t* ctx, int64_t* n);

/* Kernel timing for measurement.  With timing on, fib_run and
 * fib_step_surrogate record a HIP event on the context's stream before and
 * after each kernel launch of these classes:
 *   FUSED:      the persistent split-step kernel (one launch per fib_run);
 *   REACTION:   reaction launches of the split schedule;
 *   DIFFUSION:  diffusion launches of the split schedule;
 *   SURROGATE:  the surrogate step kernel (network or closed-form predictor);
 *   FALLBACK:   the plain Heun pair on the rejected nodes.
 * (Adaptive runs are not timed.)  Completed pairs are read back without
 * blocking once more than a few thousand are outstanding. */
enum { FIB_KT_FUSED = 0, FIB_KT_REACTION = 1, FIB_KT_DIFFUSION = 2, FIB_KT_SURROGATE = 3,
       FIB_KT_FALLBACK = 4, FIB_KT_COUNT = 5 };

/* Turns kernel timing on (enable != 0) or off and clears the sums.
 * Blocking. */
int fib_set_kernel_timing(fib_t* ctx, int32_t enable);

/* Summed device time (ms, host) and number of timed launches of kernel
 * class `cls` since timing was last turned on.  Blocking. */
int fib_kernel_time(fib_t* ctx, int32_t cls, double* ms, int64_t* launches);

/* Predictors of the surrogate step.  NETWORK is the trained network
 * (fib_set_surrogate); ZERO and EULER are closed-form guesses that go
 * through the same corrector, acceptance test and fallback:
 *   ZERO:  du = 0, so the first iterate is dt G(y, I) and a node is
 *          accepted only if its whole increment is within the tolerance;
 *   EULER: du = dt G(y, I) (one more right-hand side), so the first iterate
 *          is the explicit-midpoint (second-order Runge-Kutta) increment
 *          and the test bounds its difference to the Euler increment.
 * They are the method without the network: the baseline that shows what the
 * network gains. */
enum { FIB_PRED_NETWORK = 0, FIB_PRED_ZERO = 1, FIB_PRED_EULER = 2 };

/* Attaches the surrogate step of fib_set_surrogate with a closed-form
 * predictor (FIB_PRED_ZERO or FIB_PRED_EULER) in place of a network:
 * acceptance |du1 - du|_k <= tol * res_scale[k] for every state (host
 * array of n_states values), the same corrector iterations, the same
 * refusals of stimulus changes and prescriptions, and the same fallback.
 * Replaces an attached network; fib_clear_surrogate detaches it.  Models
 * Hodgkin-Huxley and ST57, Strang splitting.  Blocking. */
int fib_set_predictor(fib_t* ctx, int32_t predictor, const float* res_scale, double tol);

/* ------------------------------------------------------------------------
 * EMG: the static bidomain step on the 3D mesh (eq. discretized_fibers_2 and
 * eq. discretized_fibers_3, the first bidomain equation eq. bidomain1 with
 * the homogeneous Neumann conditions of eq. monodomain_bc):
 *   V_3D = P V_m,   K_{sigma_i + sigma_e} phi_e = -K_{sigma_i} V_3D.
 * The context's fibers form a bundle of nx x ny parallel fibers of equal
 * length n along z, fiber f = j nx + i at (i hx, j hy); the 3D mesh of
 * trilinear hexahedra has the fiber nodes 0, m, 2m, ... as its nodes
 * (nz = (n - 1) / m + 1 layers, layer spacing m h), so P is the injection
 * of those nodes.  3D node (i, j, k) has index (k ny + j) nx + i.
 * sigma_i = sigma_i e_z e_z^T (conduction along the fibers only) and
 * sigma_e = diag(sigma_et, sigma_et, sigma_el).
 * ------------------------------------------------------------------------ */
typedef struct fib_emg fib_emg_t;

typedef struct {
  int32_t nx, ny;    /* fibers along x and y (each >= 2); n_fibers = nx ny */
  int32_t stride;    /* m >= 1; (n - 1) must be a multiple of m and (n - 1) / m >= 1 */
  double hx, hy;     /* fiber spacing (cm, > 0) */
  double sigma_i;    /* intracellular conductivity along the fibers (mS/cm, > 0) */
  double sigma_el;   /* extracellular conductivity along the fibers (mS/cm, > 0) */
  double sigma_et;   /* extracellular conductivity across the fibers (mS/cm, > 0) */
} fib_emg_params;

/* Sets up the EMG solve for a context (which must outlive it); FIB_EINVAL
 * if the fibers do not form the bundle described above.  phi_e starts at
 * zero.  Every model (V_m is state row 0 of each). */
int fib_emg_create(fib_t* ctx, const fib_emg_params* p, fib_emg_t** out);
void fib_emg_destroy(fib_emg_t* emg);
int fib_emg_dims(const fib_emg_t* emg, int32_t* nx, int32_t* ny, int32_t* nz);

/* One static bidomain solve from the context's current V_m, on its stream:
 * right-hand side b = -K_{sigma_i} P V_m (V_m taken relative to the
 * resting potential, which K_{sigma_i} annihilates), projected to zero mean;
 * then conjugate gradients with the diagonal of K_{sigma_i + sigma_e} as
 * preconditioner, started from the last phi_e, with the residual kept at
 * zero mean (the range of the singular Neumann operator) in every
 * iteration, until ||r||_2 <= tol ||b||_2 or max_iter iterations; phi_e is
 * returned to zero mean.  FP32 vectors, FP64 reductions; tolerances down to
 * about 1e-9 are reachable.  iters and rel_res (nullable)
 * receive the iterations taken and ||r|| / ||b|| (0 if b = 0).  Blocking. */
int fib_emg_solve(fib_emg_t* emg, double tol, int32_t max_iter, int32_t* iters,
                  double* rel_res);

/* phi_e (mV) of the last solve into a host array of nx ny nz values. */
int fib_emg_get_phi(fib_emg_t* emg, double* phi, int64_t n);

/* The right-hand side -K_{sigma_i} P V_m of the last solve, before its
 * zero-mean projection, into a host array of nx ny nz values. */
int fib_emg_get_rhs(fib_emg_t* emg, double* rhs, int64_t n);

/* ------------------------------------------------------------------------
 * Measured ceilings of the current device, the empirical side of the
 * roofline (the thesis measures its CPU's peak performance with a
 * microbenchmark rather than taking the data sheet's, section "Roofline
 * Model").  One probe kernel per call, filling every compute unit, timed
 * with HIP events on the null stream after a warm-up launch:
 *   FMA:  FP32 fused multiply-adds in the two-operand (VOP2) encoding
 *         (lane operations per second);
 *   FMA_VOP3: the same in the three-operand (VOP3) encoding, which issues
 *         at half the VOP2 rate on gfx950;
 *   EXP:  v_exp_f32 (lane operations per second);
 *   RCP:  v_rcp_f32 (lane operations per second);
 *   LOG:  v_exp_f32 and v_log_f32 alternating in one chain, both counted
 *         (with the EXP rate the two separate);
 *   COPY: device-to-device copy of `bytes` (1 MiB .. 64 GiB), bytes read
 *         plus bytes written per second;
 *   MFMA_BF16: FLOP/s of v_mfma_f32_16x16x32_bf16.
 * `bytes` is ignored except for COPY.  Allocates and frees its own device
 * buffers; synchronizes the device.  rate (host) receives the result. */
enum { FIB_PROBE_FMA = 0, FIB_PROBE_EXP = 1, FIB_PROBE_RCP = 2, FIB_PROBE_LOG = 3,
       FIB_PROBE_COPY = 4, FIB_PROBE_MFMA_BF16 = 5, FIB_PROBE_FMA_VOP3 = 6 };
int fib_probe(int32_t kind, int64_t bytes, double* rate);

#ifdef __cplusplus
}
#endif

#endif /* FIB_H */
