// Internal interface between the host runtime (idm_api.hip) and the kernels
// (idm_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "idm.h"
#include <stdint.h>

namespace idmx {

// Slot flags: a bundle is threads*per_thread consecutive slots holding whole
// lanes (head -> tail) followed by padding; a lane longer than a bundle is cut
// into pieces, a piece after the first opening its bundle without a head flag.
// A halo tile (one lane's vehicles, see the tile kernels) also marks the
// vehicles whose results it owns.
enum : uint8_t { SLOT_HEAD = 1u, SLOT_TAIL = 2u, SLOT_VALID = 4u, SLOT_OWNED = 8u };

// Everything a simulation kernel reads, passed by value as the kernel argument.
struct SimArgs {
    int64_t n;          // vehicles N
    int32_t n_steps;    // S
    int32_t K;          // checkpoint interval / backward block length
    float dt, inv_dt, a_min, gap_floor;

    // bundle layout (device, owned by the plan)
    const int32_t *slot_gidx;   // [n_bundles * C], -1 = padding
    const uint8_t *slot_flags;  // [n_bundles * C]
    int32_t n_bundles;

    // inputs
    const float *v0, *T, *a, *b, *s0, *len;
    const double *p0;
    const float *v_init;

    // forward outputs
    float *traj_d, *traj_v;   // nullable
    float *ckpt;              // [nblk][2][N], nullable in forward

    // backward upstream
    const float *gd, *gv;     // nullable, [(S+1)*N]
    const float *zero;        // >= 1 zero word (plan-owned), read in place of absent inputs
    const float *target;      // nullable, [n_obs][N]
    int32_t n_obs, obs_first, obs_stride;
    double inv_count;         // 1 / (n_obs * N)
    double two_inv_count;     // 2 / (n_obs * N)

    // backward outputs
    double *g_prm;            // [5][N]
    double *g_p0, *g_v0;      // [N]
    double *loss_part;        // [n_bundles]

    // forward diagnostics (nullable): per bundle, the number of (vehicle,
    // step) evaluations whose gap was at or below gap_floor, and the number
    // of vehicles whose final state is not finite
    uint64_t *diag;           // [n_bundles][2]

    // pieces of lanes longer than a bundle (null when there are none).  A
    // bundle with bnd_in[b] = j >= 0 starts with a piece whose leader is the
    // last vehicle of the previous piece: that leader's state at step k is
    // ext_state[j*(S+1) + k], and the piece head's adjoint contribution to it
    // goes to ext_adj[j*S + k].  A bundle with bnd_out[b] = j >= 0 ends with
    // that leader: it writes ext_state and reads ext_adj of boundary j.
    const int32_t *bnd_in, *bnd_out;  // [n_bundles], -1 = none
    float2 *ext_state;                // [n_boundaries][S+1]
    float2 *ext_adj;                  // [n_boundaries][S]

    // halo tiles: the launch runs steps [k_lo, k_hi) (the forward upwards, the
    // backward downwards).  The backward carries each vehicle's adjoint of
    // (d, v) between launches through tc_in / tc_out ([2][N], two buffers
    // used alternately, since a tile reads its halo's entries while their
    // owners write the next ones), and the owned vehicles' running sums
    // through t_gp0 ([N], FP32) and t_acc ([6][N]: the five FP64 parameter
    // sums, then the FP64 loss).
    int32_t k_lo, k_hi;
    const float *tc_in;
    float *tc_out;
    float *t_gp0;
    double *t_acc;
};

struct AdamArgs {
    int64_t n;
    float *u, *m, *v, *params;
    const double *grad;   // [5][N]
    const int32_t *step;  // device counter (already incremented for this step)
    int32_t *step_rw;     // same counter, written by the initialisation kernel
    float lo[5], hi[5];
    float lr0, lr1;
    int32_t lr_steps;
    float beta1, beta2, eps;
    int32_t raw;          // 1: Adam on the physical parameters (moments of dL/dtheta)
};

// Ego-only reconstruction (one vehicle per trajectory, per-step free gap and
// speed difference to an unsimulated leader).
struct EgoArgs {
    int64_t n;          // trajectories N
    int32_t n_steps;    // S
    int32_t K;          // checkpoint interval
    float dt, inv_dt, a_min, gap_floor;
    const float *v0, *T, *a, *b, *s0;  // [N]
    const float *gap, *dv;             // [S][N]
    const float *v_init;               // [N]
    float *traj_p, *traj_v, *traj_a;   // nullable: [(S+1)][N], [(S+1)][N], [S][N]
    float *ckpt;                       // [nblk][2][N]
    // backward
    const int32_t *obs_off;            // [N+1]
    const int32_t *obs_step;           // [M], non-decreasing within a trajectory
    const float *obs_pos;              // [M]
    double *g_prm;                     // [5][N]
    float *g_gap, *g_dv;               // [S][N]
    double *g_v0;                      // [N], nullable
    double *loss_part;                 // [N] summed absolute error per trajectory
};

struct EgoAdamArgs {
    int64_t n, sn;                     // N, S*N
    float *params;                     // [5][N] physical parameters
    float *gap, *dv;                   // [S][N]
    float *m, *v;                      // [5N + 2SN] moments
    const double *g_prm;               // [5][N]
    const float *g_gap, *g_dv;         // [S][N]
    const int32_t *step;               // 1-based step after the finalize kernel
    int32_t *step_rw;
    float lo[5], hi[5];
    float lr0, lr1;
    int32_t lr_steps;
    float beta1, beta2, eps;
};

using KernelFn = const void *;

// Lookup of compiled kernel instantiations; nullptr when not instantiated.
// edge_cached: the instantiation whose bundle-edge waves store both
// trajectory rows through the cache (for launches that write both rows and
// fill the chip); otherwise every store is streamed.
KernelFn forward_kernel(int mode, int per_thread, int threads, bool pieces, bool edge_cached);
// Backward kernel for a register block KB and checkpoint interval K (the
// stash variant when K = 2 KB and one is instantiated for the shape); `dense`
// selects the variant that reads dense upstream gradients.
KernelFn backward_kernel(int mode, int per_thread, int threads, int KB, int K, bool dense,
                         bool pieces);
// Backward that reads every step's states from the forward's stored
// trajectory (whole lanes only).
KernelFn backward_stored_kernel(int mode, int per_thread, int threads, bool dense);
// Halo-tile forward and backward (one vehicle per thread; nullptr when the
// work-group size has no instantiation).
KernelFn forward_tiled_kernel(int mode, int threads);
KernelFn backward_tiled_kernel(int mode, int threads, bool dense);

// Launch helpers (return the HIP error of the launch).
hipError_t launch_sim(KernelFn fn, int grid, int threads, const SimArgs &a, hipStream_t s);
hipError_t launch_loss_finalize(const double *part, int32_t n_part, double scale, double *out,
                                hipStream_t s);
hipError_t launch_diag_finalize(const uint64_t *part, int32_t n_part, int64_t *out, hipStream_t s);
hipError_t launch_fit_finalize(const double *part, int32_t n_part, double scale,
                               int32_t *step, double *hist, int32_t hist_len, hipStream_t s);
hipError_t launch_adam(const AdamArgs &a, hipStream_t s);
// Ego-only reconstruction kernels (block = one checkpoint interval K for the
// backward; K must be 8, 16 or 32).
hipError_t launch_ego_forward(int mode, const EgoArgs &a, hipStream_t s);
hipError_t launch_ego_backward(int mode, const EgoArgs &a, hipStream_t s);
hipError_t launch_ego_adam(const EgoAdamArgs &a, hipStream_t s);
hipError_t launch_ego_fit_init(const EgoAdamArgs &a, const float *init5, float gap0, float dv0,
                               hipStream_t s);
hipError_t launch_ego_match_steps(const double *t, int32_t m, double dt, int32_t n_steps,
                                  int32_t *step_out, hipStream_t s);
hipError_t launch_ego_initial_speed(const int32_t *off, const double *t, const float *pos,
                                    int64_t n, float *v_out, hipStream_t s);
hipError_t launch_copy(const void *src, void *dst, int64_t n16, int grid, hipStream_t s);
hipError_t launch_params_from_u(const AdamArgs &a, hipStream_t s);
hipError_t launch_fit_init(const AdamArgs &a, const float *init, hipStream_t s);
hipError_t launch_fit_init_u(const AdamArgs &a, const float *u_rows, int ld, hipStream_t s);
hipError_t launch_observe(const float *traj_d, const double *p0, const float *noise, int n_obs,
                          int obs_first, int obs_stride, int64_t N, float *out, hipStream_t s);
hipError_t launch_lane_loss(const float *traj_d, const double *p0, const float *target, int n_obs,
                            int obs_first, int obs_stride, int64_t N, const int32_t *lane_off,
                            int n_lanes, double *out, hipStream_t s);
hipError_t launch_select_by_lane(const double *la, const double *lb, const int32_t *lane_of,
                                 const float *pa, const float *pb, int64_t N, float *out,
                                 int32_t *chose_a, hipStream_t s);

// Shared error reporting (idm_last_error) and plan accessors for the MLP code.
idm_status set_error(idm_status st, const char *msg);
const uint8_t *plan_head_flags(const idm_plan *p);  // device [N]: 1 = lane head
int64_t plan_vehicles(const idm_plan *p);
int32_t plan_steps(const idm_plan *p);
float plan_dt(const idm_plan *p);

}  // namespace idmx
