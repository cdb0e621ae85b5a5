/*
 * idm.h -- C ABI of the MI355X (gfx950) differentiable IDM traffic simulator.
 *
 * Method: "Gradient-based Trajectory Optimization with Parallelized
 * Differentiable Traffic Simulation" (arXiv 2412.16750).
 *   - Sec. III-A, Eqs. 1-2: each vehicle's acceleration follows the Intelligent
 *     Driver Model from its own speed and the gap / speed difference to the
 *     vehicle directly ahead in its lane (its leader h(i)).
 *   - Sec. III-A, Eq. 3: explicit Euler update, position with the old speed.
 *   - Sec. III-B, Fig. 3: all vehicles of a frame are updated synchronously
 *     from the same frame's state.
 *   - Sec. III-C: optional softplus lower bounds (s_opt >= 0 and
 *     a >= max(-v/dt, a_min)), which keep speeds non-negative.
 *   - Sec. IV-A: parameters are fitted by gradient descent on a trajectory
 *     loss against observed positions; Adam with box constraints.
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE pointers owned by the caller unless the name ends in
 *     _host.  The library never frees or retains caller memory.
 *   - Vehicles are grouped in lanes given by CSR offsets; inside a lane they
 *     are ordered head -> tail (the leader of vehicle i is i-1 unless i is the
 *     first vehicle of its lane, which drives on a free road).
 *   - Per-vehicle arrays have N entries; per-step arrays are step-major
 *     [(n_steps+1) * N], element k*N + i being vehicle i at step k.
 *   - Positions are handled as FP64 initial positions p0 plus FP32
 *     displacements d_k = p_k - p0.
 *   - Parameter blocks are ordered (v0, T, a, b, s0) = (v_targ, T_pref,
 *     a_max, a_pref, s_min) in the paper's notation.
 *   - All compute calls are asynchronous on `stream` (a hipStream_t passed as
 *     void*), allocate nothing, synchronise nothing, and can be captured in a
 *     HIP graph.  Arguments are validated before any launch; on error nothing
 *     is launched, the status is returned and idm_last_error() describes it.
 *   - Nothing throws across this boundary.
 */
#ifndef IDM_H
#define IDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IDM_OK = 0,
    IDM_ERR_INVALID_ARG = -1, /* null pointer, non-positive size, NaN, ... */
    IDM_ERR_LAYOUT = -2,      /* lane offsets not monotone / not covering N, layout too large */
    IDM_ERR_UNSUPPORTED = -3, /* a value the kernels do not implement (e.g. delta != 4) */
    IDM_ERR_WORKSPACE = -4,   /* workspace missing or too small */
    IDM_ERR_HIP = -5          /* a HIP runtime call failed; message has the HIP error */
} idm_status;

/* Velocity bound. */
enum {
    IDM_BOUND_SOFTPLUS = 0, /* Sec. III-C: s* = softplus(s_opt); a* = a_lb + softplus(a - a_lb) */
    IDM_BOUND_CLAMP = 1     /* textbook IDM, speed clamped: v' = max(v + dt*a, 0) */
};

/* Largest N: per-step rows of N floats are addressed with 32-bit byte offsets. */
#define IDM_MAX_VEHICLES (1 << 29)
/* Largest S: per-boundary rows of S + 1 steps are addressed with 32-bit byte offsets. */
#define IDM_MAX_STEPS (1 << 27)

/* The simulation problem (Sec. III-A): lanes, step count and constants. */
typedef struct {
    int32_t n_vehicles;               /* 1 <= N <= IDM_MAX_VEHICLES */
    int32_t n_lanes;                  /* L >= 1 */
    int32_t n_steps;                  /* 0 <= S <= IDM_MAX_STEPS Euler steps of length dt */
    int32_t ckpt_every;               /* K: checkpoint interval of the forward; the backward
                                         sweeps each K-step block from its last register
                                         sub-block (see idm_tuning.block) to its first;
                                         0 = let the library choose */
    float dt;                         /* > 0, seconds */
    float delta;                      /* free-road exponent; only 4 is implemented */
    float a_min;                      /* maximum deceleration bound (< 0), e.g. -10 */
    float gap_floor;                  /* gap used in (s/gap)^2 is max(gap, gap_floor) >= 0 */
    int32_t bound;                    /* IDM_BOUND_* */
    const int32_t *lane_offsets_host; /* [L+1], offsets[0] = 0, offsets[L] = N, non-decreasing */
} idm_problem;

/* Launch shape.  Zero fields mean "choose".  A work-group of `threads`
 * threads owns a bundle of `threads * per_thread` consecutive vehicle slots
 * holding whole lanes.  A lane longer than a bundle is cut into pieces of one
 * bundle each (plus a remainder); piece j runs in launch level j, after piece
 * j-1 in the forward and before it in the backward, and the two exchange the
 * boundary vehicle's state and adjoint contribution at every step through the
 * workspace.  Results do not depend on the cut (the same arithmetic in the
 * same order).  The default is 1024 threads x 1 for lanes above 1024. */
typedef struct {
    int32_t threads;    /* 64, 128, 256, 512 or 1024 (576, 640, 768 with halo tiles) */
    int32_t per_thread; /* vehicles per thread: 1, 2 or 4 */
    int32_t ckpt_every; /* K, overrides the problem's K when > 0 */
    int32_t grid;       /* >0: persistent grid of that many work-groups walking the bundle
                           list; 0: one work-group per bundle */
    int32_t block;      /* backward register block KB: 8, 16 or 32 with 1 or 2 vehicles per
                           thread, 4 or 8 with 4; must divide K; 0 = choose.  With K = 2 KB
                           on (512 or 1024 threads x 1, 512 x 2, 256 x 4 with KB = 8) the
                           backward keeps the lower sub-block's states in LDS and computes
                           every state of a block once */
    int32_t store_states; /* 1: the forward keeps every step's displacements and speeds in
                           the workspace (8 (S+1) N bytes, no checkpoints) and the backward
                           reads them instead of recomputing them from checkpoints (the
                           kernel of idm_sim_backward_stored; same results bit for bit, K
                           then only groups the FP32 gradient sums).  Fastest where a step's
                           latency, not the chip's throughput, sets the time (few lanes,
                           e.g. a fit of 100 lanes); whole lanes only (a plan whose bundles
                           would cut a lane is IDM_ERR_UNSUPPORTED).  0: checkpoints.
                           2: start with checkpoints and let idm_plan_autotune time both
                           backwards (the kept states only where the workspace it is given
                           holds them) and keep the faster */
    int32_t tile_steps;   /* J > 0: halo tiles (needs store_states 1, one vehicle per thread and
                           explicit threads of 256, 512, 576, 640, 768 (those three for tiles
                           only) or 1024; J even, a multiple of K and below threads; grid 0).  A
                           lane of n > threads vehicles is cut into the fewest tiles of at most
                           threads - 1 slots that hold it, ceil((n - J) / (threads - 1 - J)), one
                           work-group each (shorter lanes share tiles of threads slots, packed
                           best-fit decreasing as bundles are), and the steps into
                           blocks of J run as successive launches: a tile also simulates up to J
                           vehicles ahead of its own in the forward and up to J behind them in
                           the backward (each direction splits the lane on its own: the lane head
                           needs no halo ahead, the tail none behind), so that information, which
                           moves one vehicle per step (Sec. III-B's synchronous update), cannot
                           reach its owned vehicles from outside within a launch.  Owned results
                           equal the whole-lane kernels' bit for bit.  For few long lanes, whose
                           work-groups leave most compute units idle.  With store_states 2 the
                           autotuner also times tile shapes; 0: whole lanes */
} idm_tuning;

/* Per-vehicle IDM parameters (Sec. III-A), FP32 [N] each, all > 0. */
typedef struct {
    const float *v0;     /* desired speed v_targ (m/s) */
    const float *T;      /* time headway T_pref (s) */
    const float *a;      /* maximum acceleration a_max (m/s^2) */
    const float *b;      /* comfortable deceleration a_pref (m/s^2) */
    const float *s0;     /* jam distance s_min (m) */
    const float *length; /* vehicle length (m); the follower subtracts its LEADER's length */
} idm_params;

/* Observed positions for the fused mean-squared trajectory loss
 * (the squared-error counterpart of Sec. IV-A, Eq. 4).  Observation j is step
 * obs_first + j*obs_stride (must be <= n_steps) for every vehicle;
 * target[j*N + i] is the observed absolute position (m), FP32.
 * L = 1/(n_obs*N) * sum_j sum_i (p0_i + d_k(i) - target[j*N+i])^2, summed in FP64. */
typedef struct {
    const float *target;
    int32_t n_obs;
    int32_t obs_first;
    int32_t obs_stride;
} idm_obs;

typedef struct idm_plan idm_plan;

/* Plan: validates the problem, packs lanes into work-group bundles and uploads
 * that small table to device memory owned by the plan (the only allocation
 * the library makes; freed by idm_plan_destroy).  `tuning` may be NULL. */
idm_status idm_plan_create(const idm_problem *problem, const idm_tuning *tuning, idm_plan **out);
idm_status idm_plan_destroy(idm_plan *plan);

/* Bytes of device workspace the caller must pass to the compute calls:
 * checkpoints ceil(S/K) * 2 * N * 4 B, per-bundle loss partials and
 * diagnostic counts (see idm_plan_diagnostics), the FP64
 * gradient buffer used by idm_fit_step and, with lanes longer than a bundle,
 * (2 S + 1) * 8 B per piece boundary.  A plan that keeps every step's states
 * holds them instead of the checkpoints (8 (S+1) N B), and with halo tiles
 * 68 N B more for the adjoints and sums carried between launches.  256-byte
 * aligned.  With piece boundaries, idm_sim_forward needs the workspace too;
 * with halo tiles it needs the workspace or both trajectory outputs. */
size_t idm_workspace_bytes(const idm_plan *plan);

/* Chosen launch shape and packing statistics. */
typedef struct {
    int32_t threads, per_thread, ckpt_every, grid;
    int32_t block;          /* backward register block KB */
    int32_t n_bundles;      /* work-group bundles */
    int32_t max_lane;       /* longest lane (vehicles) */
    int64_t n_slots;        /* bundles * threads * per_thread */
    double fill;            /* N / n_slots */
    int32_t n_levels;       /* launches per pass: 1 + most extra pieces of one lane */
    int32_t n_boundaries;   /* piece boundaries of lanes longer than a bundle */
    int32_t autotune_cached; /* 1: the last idm_plan_autotune took its shape from the cache */
    int32_t store_states;   /* 1: every step's states are kept (idm_tuning.store_states 1, or
                               2 after the autotuner chose them) */
    int32_t tile_steps;     /* J of halo tiles (n_bundles then counts tiles), 0: whole lanes */
} idm_plan_info;
idm_status idm_plan_get_info(const idm_plan *plan, idm_plan_info *out);

/* Host-only checks (no device needed, nothing allocated): validate a problem
 * and tuning exactly as idm_plan_create does, and report the launch shape,
 * bundle statistics and workspace size it would get (info and
 * workspace_bytes are nullable). */
idm_status idm_problem_check(const idm_problem *problem, const idm_tuning *tuning,
                             idm_plan_info *info, size_t *workspace_bytes);

/* Host-only: the bundle layout idm_plan_create would upload.  Slot s of
 * bundle b is element b*threads*per_thread + s; slot_vehicle_host receives the
 * vehicle index (-1 = padding) and slot_flags_host bit 0 = lane head, bit 1 =
 * lane tail, bit 2 = occupied.  Both arrays must hold `capacity` >= n_slots
 * entries (see idm_problem_check), else IDM_ERR_INVALID_ARG.  With halo tiles
 * (tile_steps > 0; n_bundles counts tiles) there are two tables of n_slots
 * each, so capacity >= 2 n_slots: the forward's (the halo ahead, then the
 * owned vehicles; bit 0 on the first slot) then the backward's (the owned
 * vehicles, then the halo behind; bit 0 only on a true lane head); bit 3
 * marks the vehicles a tile owns. */
idm_status idm_problem_layout(const idm_problem *problem, const idm_tuning *tuning,
                              int32_t *slot_vehicle_host, uint8_t *slot_flags_host,
                              int64_t capacity);

/* Host-only: per bundle (in the order of idm_problem_layout), the piece
 * boundary whose leader state the bundle's first slot reads (bnd_in, -1 if
 * its first slot is a lane head or padding), the boundary its last slot
 * leads (bnd_out, -1 if none) and its launch level.  A piece's head slot
 * carries no head flag; only a lane's first and last vehicles are flagged.
 * Arrays hold `capacity` >= n_bundles entries, else IDM_ERR_INVALID_ARG. */
idm_status idm_problem_bundles(const idm_problem *problem, const idm_tuning *tuning,
                               int32_t *bnd_in_host, int32_t *bnd_out_host, int32_t *level_host,
                               int64_t capacity);

/* Forward simulation (Eqs. 1-3 with the chosen bound, Sec. III-B update
 * order), all n_steps in one launch per launch level (one level unless lanes
 * are longer than a bundle).
 *   p0      [N] FP64 initial positions;  v_init [N] FP32 initial speeds.
 *   traj_d  [(S+1)*N] FP32 displacement p_k - p0 (nullable: not written).
 *   traj_v  [(S+1)*N] FP32 speeds (nullable).
 *   workspace: receives the checkpoints the backward pass needs (may be NULL
 *   when no backward will follow and no lane is cut into pieces; with pieces
 *   a NULL workspace is IDM_ERR_WORKSPACE). */
idm_status idm_sim_forward(idm_plan *plan, const idm_params *prm, const double *p0,
                           const float *v_init, float *traj_d, float *traj_v, void *workspace,
                           void *stream);

/* Runtime anomalies of the most recent forward pass that wrote `workspace`
 * for this plan (idm_sim_forward with a workspace, idm_fit_step,
 * idm_fit_run, idm_step_graph_launch).  The gap that enters (s* / gap)^2
 * (Sec. III-A, Eq. 2) is max(gap, gap_floor) so that the interaction term
 * stays finite when vehicles touch or overlap; the forward counts how often
 * that floor was active.  counts_out (DEVICE int64[2]) receives
 *   [0] the number of (vehicle, step) evaluations with gap <= gap_floor
 *       (a lane head never counts: it drives on a free road),
 *   [1] the number of vehicles whose state (displacement or speed) was not
 *       finite at some step (a non-finite speed makes every later
 *       displacement non-finite, so the final state decides).
 * The forward writes per-bundle counts into the workspace with plain stores;
 * this call sums them in a fixed order (one small kernel, asynchronous on
 * `stream`, graph-capturable).  A workspace no forward has written gives
 * meaningless counts; a forward called with a NULL workspace writes none. */
idm_status idm_plan_diagnostics(idm_plan *plan, const void *workspace, int64_t *counts_out,
                                void *stream);

/* Reverse-mode gradient of a scalar loss L with respect to the five
 * parameters and the initial state (the paper differentiates the same
 * simulation, Sec. III-B).  Must follow idm_sim_forward with the same inputs
 * and workspace (it recomputes each K-step block from the checkpoints).
 * Upstream gradient = any combination of:
 *   grad_traj_d [(S+1)*N] FP32 dL/dd_k (= dL/dp_k), nullable;
 *   grad_traj_v [(S+1)*N] FP32 dL/dv_k, nullable;
 *   obs: fused mean-squared trajectory loss (see idm_obs), nullable.
 * Outputs (overwritten, FP64): grad_params [5*N] (v0, T, a, b, s0 blocks),
 * grad_p0 [N] = dL/dp0 and grad_v0 [N] = dL/dv(0).  grad_p0 treats the dense
 * upstream grad_traj_d as acting on the displacements at fixed p0 (so it
 * reaches p0 only through the gaps), and the fused loss as acting on the
 * absolute positions p0 + d_k (gap terms plus its direct term).  loss_out (device FP64
 * scalar, nullable) receives the fused loss (0 if obs is NULL).  Per-vehicle
 * gradients are summed over time in FP64 in a fixed order; no atomics, so
 * results are bitwise reproducible. */
idm_status idm_sim_backward(idm_plan *plan, const idm_params *prm, const double *p0,
                            const float *v_init, const float *grad_traj_d,
                            const float *grad_traj_v, const idm_obs *obs, double *grad_params,
                            double *grad_p0, double *grad_v0, double *loss_out, void *workspace,
                            void *stream);

/* The gradient of idm_sim_backward computed from the forward's stored
 * trajectory instead of checkpoints (the same reverse pass through the
 * simulation of Sec. III-B, with every state kept).  traj_d and traj_v
 * [(S+1)*N] FP32 are the displacements and speeds idm_sim_forward wrote for
 * the same plan and inputs (both required, read only; that forward needs no
 * workspace, since no checkpoints are read).  Each step's states are read
 * instead of recomputed, which removes the recomputation's third of the
 * backward's arithmetic for 8 more bytes read per vehicle-step, and keeps the
 * 8 (S+1) N bytes of trajectory in device memory in place of the checkpoints.
 * grad_traj_d, grad_traj_v, obs, the outputs and their meaning as in
 * idm_sim_backward; the workspace (idm_workspace_bytes) receives only the
 * loss partials.  Results equal idm_sim_backward's bit for bit for the same
 * plan (the same K-step blocks of FP32 gradient sums).  A plan that cuts
 * lanes into pieces (idm_plan_info.n_boundaries > 0) is IDM_ERR_UNSUPPORTED:
 * use idm_sim_backward. */
idm_status idm_sim_backward_stored(idm_plan *plan, const idm_params *prm, const double *p0,
                                   const float *traj_d, const float *traj_v,
                                   const float *grad_traj_d, const float *grad_traj_v,
                                   const idm_obs *obs, double *grad_params, double *grad_p0,
                                   double *grad_v0, double *loss_out, void *workspace,
                                   void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * gradient of idm_sim_backward with no workspace argument.  One call runs the
 * forward (checkpoints only, no trajectory) and then the backward, the same
 * kernels as idm_sim_forward + idm_sim_backward on a caller workspace, with
 * the library's static device scratch array in that workspace's place; the
 * outputs (grad_params, grad_p0, grad_v0, loss_out, same layout and meaning
 * as idm_sim_backward) are bitwise equal to that pair's.
 *   - Allocates nothing: no hipMalloc, hipFree or allocating library call.
 *     The scratch array, IDM_STATIC_SCRATCH_BYTES (256 MiB) per GPU, is part
 *     of the library's device code and is held until the process ends; its
 *     address is looked up once per device (first call on that device).
 *   - A plan whose workspace (idm_workspace_bytes) exceeds the array is
 *     rejected with IDM_ERR_WORKSPACE before anything is launched (the
 *     2000 x 1000-vehicle, 100-step, K = 32 problem needs 176 MiB and fits).
 *   - Every call on one GPU shares that GPU's array and leaves its contents
 *     there; nothing in it needs to start at zero (each region the kernels
 *     read is written earlier in the same call).  Calls that overlap on one
 *     GPU (two streams, two threads) race on the array: serialize them.
 *   - idm_plan_diagnostics cannot read this call's counts (the scratch is
 *     not a caller workspace). */
#define IDM_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
idm_status idm_sim_backward_noalloc(idm_plan *plan, const idm_params *prm, const double *p0,
                                    const float *v_init, const float *grad_traj_d,
                                    const float *grad_traj_v, const idm_obs *obs,
                                    double *grad_params, double *grad_p0, double *grad_v0,
                                    double *loss_out, void *stream);

/* One gradient step of the trajectory fit (Sec. IV-A): forward (checkpoints
 * only), fused MSE loss and backward, then Adam on NORMALISED parameters
 * u = (theta - lo) / (hi - lo) followed by projection of u onto [0, 1] (the
 * paper's box constraints), or, with raw_units = 1, Adam on the physical
 * parameters theta themselves with the learning rate in their own units
 * followed by projection onto [lo, hi] (the paper's fitting, Sec. IV-A and
 * Sec. V-B3).  The physical parameters params[5*N] are rewritten after the
 * step and are what the simulation reads; u always holds
 * (theta - lo) / (hi - lo).
 * All state lives in device memory, so a call can be captured in a HIP graph
 * and replayed (see idm_fit_run). */
typedef struct {
    float *u;              /* [5*N] normalised parameters, updated */
    float *m;              /* [5*N] Adam first moment (of dL/du, or of dL/dtheta with raw_units), updated */
    float *v;              /* [5*N] Adam second moment (same variable), updated */
    float *params;         /* [5*N] physical parameters (v0, T, a, b, s0 blocks), rewritten */
    const float *length;   /* [N] vehicle lengths */
    int32_t *step;         /* device int32: Adam step counter t (0 before the first step), updated */
    double *loss_hist;     /* device [hist_len] FP64: loss of step t goes to min(t, hist_len-1) */
    int32_t hist_len;      /* >= 1 */
    float lo[5], hi[5];    /* box per parameter kind, hi > lo */
    float lr0, lr1;        /* learning rate, linear from lr0 (t=0) to lr1 (t >= lr_steps) */
    int32_t lr_steps;      /* >= 1 */
    float beta1, beta2, eps;
    int32_t raw_units;     /* 0: Adam on u; 1: Adam on theta (lr in the parameters' units) */
} idm_fit_state;

/* Start a fit from physical parameters init_params [5*N] (device FP32):
 * u = clamp((theta - lo)/(hi - lo), 0, 1), Adam moments 0, step counter 0,
 * params rewritten from u.  One kernel; graph-capturable. */
idm_status idm_fit_init(idm_plan *plan, const idm_fit_state *st, const float *init_params,
                        void *stream);

/* Start a fit from normalised parameters given as rows: u of vehicle i and
 * kind p at u_rows[i*ld + p] (ld >= 5; e.g. the MLP output with ld =
 * IDM_MLP_OUT_PAD), clamped to [0, 1]; moments and step counter reset. */
idm_status idm_fit_init_normalized(idm_plan *plan, const idm_fit_state *st, const float *u_rows,
                                   int32_t ld, void *stream);

idm_status idm_fit_step(idm_plan *plan, const idm_fit_state *st, const double *p0,
                        const float *v_init, const idm_obs *obs, void *workspace, void *stream);

/* n_iters fit steps: the first call for a given argument set captures one
 * step in a HIP graph owned by the plan; every iteration is a graph replay. */
idm_status idm_fit_run(idm_plan *plan, const idm_fit_state *st, const double *p0,
                       const float *v_init, const idm_obs *obs, int32_t n_iters,
                       void *workspace, void *stream);

/* Forward + backward as one HIP graph (captured on first use for a given
 * argument set, then replayed): the batched launch for many independent
 * lanes.  Arguments as in idm_sim_forward / idm_sim_backward, except that a
 * plan keeping every step's states (store_states 1) keeps them in traj_d /
 * traj_v where those are given, instead of in the workspace, and the step's
 * backward reads them there (no copy between the two); a later
 * idm_sim_backward on that workspace does not see them. */
typedef struct {
    idm_params prm;
    const double *p0;
    const float *v_init;
    float *traj_d, *traj_v;
    const float *grad_traj_d, *grad_traj_v;
    const float *obs_target; /* NULL: no fused loss */
    int32_t n_obs, obs_first, obs_stride;
    double *grad_params, *grad_p0, *grad_v0, *loss_out;
    void *workspace;
} idm_step_args;
idm_status idm_step_graph_launch(idm_plan *plan, const idm_step_args *args, void *stream);

/* Autotuner: times forward + backward of every candidate launch shape
 * (threads x per_thread x KB, with K the problem's or, left free
 * (ckpt_every = 0 at plan creation), KB and 2 KB where the LDS stash exists;
 * with store_states 2 also the kept-state backward and halo tiles) whose
 * lanes fit and whose workspace fits in `workspace_bytes`, as the best of
 * three batches of `reps` replays of the candidate's captured forward +
 * backward graph (after `reps` untimed ones), on the real inputs, and
 * switches the plan to the fastest.  The choice
 * is cached for the process, keyed by the sorted lane sizes (the lane-size
 * histogram), S, the bound mode, the kind of upstream gradient, a fixed K
 * and the device's compute-unit count: a later call for an equal problem
 * takes the cached shape without timing (idm_plan_info.autotune_cached = 1)
 * when its workspace fits.  To keep a choice across processes, read it with
 * idm_plan_get_info and pass it as idm_tuning to idm_plan_create.  Shapes whose backward spills registers are timed only
 * when no other shape holds the longest lane (lanes above 2048 vehicles).  Synchronises `stream`.  Results of the timed runs are
 * discarded (they overwrite the output buffers).  Any graph captured by the
 * plan is dropped. */
idm_status idm_plan_autotune(idm_plan *plan, const idm_step_args *args, size_t workspace_bytes,
                             int32_t reps, void *stream);

/* Observations from a simulated trajectory (synthetic data generation):
 * target_out[j*N + i] = p0[i] + traj_d[(obs_first + j*obs_stride)*N + i]
 * + noise[j*N + i] (noise nullable), FP32; observed steps must be <= n_steps. */
idm_status idm_observe(idm_plan *plan, const float *traj_d, const double *p0, const float *noise,
                       int32_t n_obs, int32_t obs_first, int32_t obs_stride, float *target_out,
                       void *stream);

/* Per-lane observed squared error of a trajectory: lane_loss[l] = sum over the
 * lane's vehicles and the observed steps of (p0 + d_k - target)^2, FP64,
 * fixed summation order. */
idm_status idm_lane_loss(idm_plan *plan, const float *traj_d, const double *p0, const idm_obs *obs,
                         double *lane_loss, void *stream);

/* Per-lane choice between two parameter sets [5*N]: every vehicle of lane l
 * takes params_a if loss_a[l] <= loss_b[l], else params_b (the warm start's
 * fallback to the cold start).  chose_a [N] (nullable) records the choice. */
idm_status idm_select_by_lane(idm_plan *plan, const double *loss_a, const double *loss_b,
                              const float *params_a, const float *params_b, float *params_out,
                              int32_t *chose_a, void *stream);

/* Plain device-to-device copy of `bytes` (multiple of 16, 16-byte aligned
 * pointers) by a streaming kernel: the measured HBM bandwidth ceiling and the
 * byte-counter calibration reference of the benchmark.  Asynchronous. */
idm_status idm_copy_bytes(void *dst, const void *src, size_t bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Learned warm start (not in the paper, whose fit starts from fixed values,
 * Sec. IV-A): a 150 -> 256 -> 256 -> 5 ReLU MLP maps the observed trajectory
 * window of a vehicle to normalised IDM parameters u in [0, 1]^5 (same boxes
 * as the fit).  BF16 MFMA GEMMs with FP32 accumulation, FP32 master weights,
 * Adam.  Feature rows are padded to IDM_MLP_IN_PAD BF16 values and outputs
 * to IDM_MLP_OUT_PAD FP32 columns (the first IDM_MLP_OUT are meaningful).
 *
 * FP32 parameter buffer (idm_mlp_param_count() floats), row-major blocks:
 *   W1 [IN_PAD x HIDDEN], b1 [HIDDEN], W2 [HIDDEN x HIDDEN], b2 [HIDDEN],
 *   W3 [HIDDEN x OUT_PAD], b3 [OUT_PAD]
 * BF16 weight copies (idm_mlp_weight_bf16_count() values, 16-byte aligned
 * buffer): W1, W2, W3 in the same layouts, back to back, then their
 * transposes W1^T [HIDDEN x IN_PAD], W2^T [HIDDEN x HIDDEN], W3^T
 * [OUT_PAD x HIDDEN] (the forward's operands).  idm_mlp_sync refreshes all of
 * them from the FP32 weights (and zeroes the Adam moments);
 * idm_mlp_train_step keeps them in sync after every update.
 * ------------------------------------------------------------------------- */
#define IDM_MLP_IN 150
#define IDM_MLP_IN_PAD 160
#define IDM_MLP_HIDDEN 256
#define IDM_MLP_OUT 5
#define IDM_MLP_OUT_PAD 16

typedef struct {
    float *params;          /* FP32 master parameters (layout above), device, 16-byte aligned */
    uint16_t *weights_bf16; /* BF16 copies of W1, W2, W3 and their transposes, device,
                               16-byte aligned (else IDM_ERR_INVALID_ARG) */
    float *adam_m, *adam_v; /* Adam moments [param_count], device (nullable for inference) */
    float lr, beta1, beta2, eps;
} idm_mlp_state;

int64_t idm_mlp_param_count(void);
int64_t idm_mlp_weight_bf16_count(void);
/* Device workspace (16-byte aligned) for gradients / train step on a batch of B rows. */
size_t idm_mlp_workspace_bytes(int64_t batch);
/* FP32 -> BF16 weight copies; zero the Adam moments if present. */
idm_status idm_mlp_sync(const idm_mlp_state *st, void *stream);
/* Window features X [N x IN_PAD] BF16 of every vehicle of the plan from its
 * observed absolute positions target [n_obs x N] (observation j at step
 * obs_first + j*obs_stride >= 1), the initial positions p0 and the lengths:
 * per observation the offset (p_j - p0)/1000 m, the finite-difference speed
 * /30 m/s (the first one from p0 at t = 0), and the gap to the observed leader
 * /50 m (200 m for a lane head); 3*n_obs <= IN_PAD, zero padded. */
idm_status idm_mlp_features(idm_plan *plan, const float *target, int32_t n_obs, int32_t obs_first,
                            int32_t obs_stride, const double *p0, const float *length,
                            uint16_t *X, void *stream);
/* Y [batch x OUT_PAD] FP32 = MLP(X), one fused launch (64 rows per
 * work-group, hidden activations kept in LDS).  X may have any alignment;
 * `workspace` is not used by the forward and may be null. */
idm_status idm_mlp_forward(const idm_mlp_state *st, const uint16_t *X, int64_t batch, float *Y,
                           void *workspace, void *stream);
/* Gradients of L = mean over batch and the 5 outputs of (Y - U)^2 (U [batch x 5]
 * FP32 normalised targets) w.r.t. every FP32 parameter, into grad_out
 * [param_count]; loss_out (device FP64, nullable) receives L. */
idm_status idm_mlp_gradients(const idm_mlp_state *st, const uint16_t *X, const float *U,
                             int64_t batch, float *grad_out, double *loss_out, void *workspace,
                             void *stream);
/* One Adam step (step number t >= 1) on the same loss; refreshes the BF16 copies. */
idm_status idm_mlp_train_step(const idm_mlp_state *st, const uint16_t *X, const float *U,
                              int64_t batch, int32_t t, double *loss_out, void *workspace,
                              void *stream);

/* Training loop state that lives in device memory, so that every step of a
 * loop is the same call and one step can be captured in a HIP graph and
 * replayed (the learning rate, the step number and the batch rows are read
 * on the device). */
typedef struct {
    int32_t *step;        /* device int32: steps done (0 before the first), incremented */
    float lr0, lr_final;  /* learning rate of step t: lr_final + (lr0 - lr_final) *
                             (1 + cos(pi (t - 1) / total_steps)) / 2, in FP64 then rounded */
    int32_t total_steps;  /* >= 1 */
    double *loss_hist;    /* device [hist_len] FP64: loss of step t at (t - 1) % hist_len */
    int32_t hist_len;     /* >= 1 */
} idm_mlp_schedule;

/* One scheduled Adam step t = *sched->step + 1 (the counter is advanced by
 * the call's last kernel); the batch is rows
 * perm[((t - 1) % (n_rows / batch)) * batch + i], i < batch, of X_all
 * [n_rows x IN_PAD] (BF16) and U_all [n_rows x 5] (FP32), gathered into Xb
 * [batch x IN_PAD] and Ub [batch x 5] (device, caller-owned); then the step of
 * idm_mlp_train_step with that t and the scheduled rate, and the loss into
 * loss_hist.  perm (device int64 [n_rows], a permutation) may be rewritten
 * between calls (one epoch per permutation); an entry outside [0, n_rows)
 * gathers a zero row.  batch <= n_rows; workspace as
 * idm_mlp_workspace_bytes(batch).  No host synchronisation, no allocation:
 * graph-capturable. */
idm_status idm_mlp_train_step_scheduled(const idm_mlp_state *st, const uint16_t *X_all,
                                        const float *U_all, int64_t n_rows, const int64_t *perm,
                                        int64_t batch, const idm_mlp_schedule *sched,
                                        uint16_t *Xb, float *Ub, void *workspace, void *stream);

/* ---------------------------------------------------------------------------
 * Ego-only reconstruction (Sec. IV-A, trajectory filtering and reconstruction).
 * Every trajectory is one vehicle starting at p(0) = 0 whose leader is not
 * simulated: its bumper-to-bumper gap G_k and speed difference D_k = v - v_h
 * at every step k are free variables next to the five parameters.  The loss
 * is the sum over trajectories and their observations of |observed position -
 * simulated position at the nearest step|.  Step-indexed arrays are
 * step-major [S][N] FP32 on the device; every pointer is device memory owned
 * by the caller unless stated otherwise.
 * ------------------------------------------------------------------------- */
typedef struct idm_ego_plan idm_ego_plan;

typedef struct {
    int32_t n_traj;     /* N trajectories, 1 <= N <= IDM_MAX_VEHICLES */
    int32_t n_steps;    /* S >= 0 steps of dt */
    int32_t ckpt_every; /* K: 8, 16 or 32 (0 = 32); checkpoint interval of the forward and
                           register block of the backward */
    float dt;           /* > 0, seconds */
    float delta;        /* only 4 is implemented */
    float a_min;        /* < 0 */
    float gap_floor;    /* >= 0 */
    int32_t bound;      /* IDM_BOUND_* */
} idm_ego_problem;

/* The fit variables: parameters [N] each (as idm_params) and the per-step
 * gap G and speed difference D [S][N] (null allowed when S = 0). */
typedef struct {
    const float *v0, *T, *a, *b, *s0;
    const float *gap, *dv;
} idm_ego_vars;

/* Observations, CSR by trajectory: trajectory i owns entries offsets[i] ..
 * offsets[i+1]-1 (offsets[0] = 0, offsets[N] = n_obs), each a simulation step
 * in 0..S (non-decreasing within a trajectory; idm_ego_match_steps maps
 * timestamps to steps) and an observed position in the p(0) = 0 frame. */
typedef struct {
    const int32_t *offsets; /* [N+1] */
    const int32_t *step;    /* [n_obs] */
    const float *pos;       /* [n_obs], m */
    int32_t n_obs;
} idm_ego_obs;

/* Validates the problem (host only) and allocates the plan (host memory). */
idm_status idm_ego_plan_create(const idm_ego_problem *pb, idm_ego_plan **out);
idm_status idm_ego_plan_destroy(idm_ego_plan *plan);
/* Caller-allocated device workspace: loss partials, fit gradients, checkpoints. */
size_t idm_ego_workspace_bytes(const idm_ego_plan *plan);
/* Nearest simulation step of each timestamp (Sec. IV-A): step_out[j] =
 * rint(t[j] / dt) in FP64, clamped to [0, n_steps]; t [m] FP64 seconds from
 * the trajectory's first observation. */
idm_status idm_ego_match_steps(const double *t, int32_t m, double dt, int32_t n_steps,
                               int32_t *step_out, void *stream);
/* Initial speed v(0) = max((P_1 - P_0) / (T_1 - T_0), 0) from each trajectory's
 * first two observations (0 with fewer than two); t FP64, pos FP32, CSR. */
idm_status idm_ego_initial_speed(const int32_t *offsets, const double *t, const float *pos,
                                 int32_t n, float *v_init_out, void *stream);
/* Forward: all S steps in one launch, one thread per trajectory; writes the
 * checkpoints into the workspace and, where non-null, positions traj_p and
 * speeds traj_v [(S+1)][N] and the acceleration of each update traj_a [S][N]
 * (CLAMP: (v' - v) / dt). */
idm_status idm_ego_forward(idm_ego_plan *plan, const idm_ego_vars *x, const float *v_init,
                           float *traj_p, float *traj_v, float *traj_a, void *workspace,
                           void *stream);
/* Backward (needs the forward's checkpoints in the workspace): gradients of
 * the summed absolute error (subgradient sign(p - obs), 0 at equality) with
 * respect to the parameters grad_params [5][N] FP64, the free variables
 * grad_gap, grad_dv [S][N] FP32 and v(0) grad_v0 [N] FP64 (nullable);
 * loss_out (FP64, nullable) receives the loss. */
idm_status idm_ego_backward(idm_ego_plan *plan, const idm_ego_vars *x, const float *v_init,
                            const idm_ego_obs *obs, double *grad_params, float *grad_gap,
                            float *grad_dv, double *grad_v0, double *loss_out, void *workspace,
                            void *stream);

/* Adam fit of the reconstruction (Sec. V-B3): parameters projected onto their
 * boxes after every step, G and D unconstrained, learning rate linear from
 * lr0 to lr1 over lr_steps steps. */
typedef struct {
    float *params;     /* [5][N] (v0, T, a, b, s0), updated in place */
    float *gap, *dv;   /* [S][N], updated in place */
    float *m, *v;      /* [5N + 2SN] Adam moments */
    int32_t *step;     /* device step counter */
    double *loss_hist; /* [hist_len] loss before each step (FP64) */
    int32_t hist_len;
    float lo[5], hi[5];
    float lr0, lr1;
    int32_t lr_steps;
    float beta1, beta2, eps;
} idm_ego_fit_state;

/* Every trajectory's parameters = init_params (v0, T, a, b, s0), every G =
 * gap0, every D = dv0, zero moments, step 0. */
idm_status idm_ego_fit_init(idm_ego_plan *plan, const idm_ego_fit_state *st,
                            const float init_params[5], float gap0, float dv0, void *stream);
/* One fit step: forward, loss + gradients, loss history, Adam. */
idm_status idm_ego_fit_step(idm_ego_plan *plan, const idm_ego_fit_state *st, const float *v_init,
                            const idm_ego_obs *obs, void *workspace, void *stream);
/* n_iters fit steps replayed from a HIP graph captured on first use. */
idm_status idm_ego_fit_run(idm_ego_plan *plan, const idm_ego_fit_state *st, const float *v_init,
                           const idm_ego_obs *obs, int32_t n_iters, void *workspace, void *stream);

/* Thread-local description of the last error (never NULL). */
const char *idm_last_error(void);

/* Library version string. */
const char *idm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* IDM_H */
