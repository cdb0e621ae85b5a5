// HIP kernels of the differentiable IDM simulator for gfx950 (MI355X).
//
// Method (arXiv 2412.16750): Sec. III-A Eqs. 1-3 (IDM acceleration from the
// gap and speed difference to the leader, explicit Euler), Sec. III-B
// (synchronous per-frame update), Sec. III-C (softplus lower bounds).  The
// reverse pass is a hand-derived adjoint of the same discrete equations.
//
// Design:
//   * A work-group owns a "bundle": threads*R consecutive slots holding whole
//     lanes (head -> tail).  Thread t owns slots t*R .. t*R+R-1, so the
//     leader of every vehicle but the thread's first one is in registers; the
//     first vehicle reads its leader (the previous thread's last vehicle)
//     from LDS.  Lanes never interact, so a work-group runs ALL time steps of
//     its bundle in one launch, with one work-group barrier per step
//     (ping-pong LDS buffers remove the second barrier).
//   * A lane longer than a bundle is cut into pieces of a whole bundle each
//     (plus a remainder).  Piece j runs in a later launch than piece j-1 in
//     the forward and an earlier one in the backward: the last vehicle of
//     piece j-1 publishes its state at every step to a boundary buffer that
//     the head of piece j reads as its leader, and the head of piece j
//     publishes its adjoint contribution to that leader at every step.  The
//     leader never depends on its follower, so each launch is complete.
//   * State is FP32 displacement d = p - p0 plus speed; the initial gap to the
//     leader g0 = p0_h - p0 - len_h is formed in FP64 once and rounded, so the
//     gap at step k is g0 + (d_h - d) without cancellation of large positions.
//   * Forward writes the trajectory (coalesced, step-major) and a checkpoint of
//     (d, v) every K steps.  Backward walks K-step blocks from last to first:
//     it reloads the block's checkpoint, recomputes the K states into
//     registers, then sweeps them in reverse.  The follower -> leader part of
//     the adjoint is a GATHER: every vehicle publishes its contribution to
//     its leader and each vehicle reads the one of its follower (slot + 1).
//     No atomics anywhere, so results are bitwise reproducible.
//   * Per-vehicle parameter gradients are summed in FP32 within a block and in
//     FP64 across blocks; the fused MSE loss is summed in FP64 per bundle and
//     reduced in a fixed order by a second kernel.
#include "idm_device.h"

#include <limits.h>
#include <math.h>

#include <type_traits>

namespace idmx {
namespace {

template <int R>
__device__ __forceinline__ void load_vehicles(const SimArgs &A, int64_t slot0, Veh (&q)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int32_t g = A.slot_gidx[slot0 + r];
        uint8_t f = A.slot_flags[slot0 + r];
        q[r].g = g;
        q[r].head = (f & SLOT_HEAD) || g < 0;
        if (g >= 0) {
            float v0 = A.v0[g], a = A.a[g], b = A.b[g];
            q[r].inv_v0 = 1.0f / v0;
            q[r].T = A.T[g];
            q[r].a = a;
            q[r].s0 = A.s0[g];
            q[r].c = 0.5f / sqrtf(a * b);
            q[r].two_a = 2.0f * a;
            q[r].fa_v0 = 4.0f * a / v0;
            q[r].i2a = 0.5f / a;
            q[r].i2b = 0.5f / b;
            if (!q[r].head) {
                double gap0 = A.p0[g - 1] - A.p0[g] - (double)A.len[g - 1];
                q[r].g0 = (float)gap0;
            } else {
                q[r].g0 = INFINITY;
            }
        } else {
            q[r].inv_v0 = 0.0f;
            q[r].T = 0.0f;
            q[r].a = 0.0f;
            q[r].s0 = 0.0f;
            q[r].c = 0.0f;
            q[r].two_a = 0.0f;
            q[r].fa_v0 = 0.0f;
            q[r].i2a = 0.0f;
            q[r].i2b = 0.0f;
            q[r].g0 = INFINITY;
        }
    }
}

// ---------------------------------------------------------------- forward

// Exchange-slot indices without masks.  Thread 0's first vehicle always opens
// a bundle, so it is a lane head (or padding, also flagged head): its gap is
// +inf and every leader term it computes is exactly zero for any finite
// leader state, so it reads its own slot instead of a missing leader.  The
// last thread reads thread 0's follower contribution, which is exactly zero
// for the same reason.  The one exception, a bundle opened by a later piece of
// a long lane, replaces both reads with the boundary buffers (ext_lead, and
// the last thread's gather in the backward).
__device__ __forceinline__ int lead_thread(int t) { return t > 0 ? t - 1 : 0; }
template <int NT>
__device__ __forceinline__ int follow_thread(int t) {
    if constexpr ((NT & (NT - 1)) == 0)
        return (t + 1) & (NT - 1);
    else
        return t + 1 < NT ? t + 1 : 0;  // halo tiles of 576, 640 or 768 threads
}

// Boundary rows of bundle `bidx` (uniform): the external leader's states and
// the adjoint contributions to it (bnd_in), and the same rows of the boundary
// this bundle's last vehicle leads (bnd_out).  Null when absent.
struct Ext {
    const float2 *lead;  // [S+1] leader state of the first vehicle
    float2 *lead_adj;    // [S]   its contribution to that leader
    float2 *tail;        // [S+1] state of the last vehicle, for the next piece
    const float2 *tail_adj;  // [S] the next piece head's contribution to it
};

template <bool CH>
__device__ __forceinline__ Ext ext_rows(const SimArgs &A, int bidx) {
    Ext x{nullptr, nullptr, nullptr, nullptr};
    if (CH && A.bnd_in) {
        const int64_t S = A.n_steps;
        const int32_t bi = A.bnd_in[bidx], bo = A.bnd_out[bidx];
        if (bi >= 0) {
            x.lead = A.ext_state + bi * (S + 1);
            x.lead_adj = A.ext_adj + bi * S;
        }
        if (bo >= 0) {
            x.tail = A.ext_state + bo * (S + 1);
            x.tail_adj = A.ext_adj + bo * S;
        }
    }
    return x;
}

// The boundary leader's states, staged 64 steps at a time through LDS by wave
// 0: lane l loads step k0 + l of the chunk after next while the current chunk
// is read from LDS, so a step never waits on memory (a wait for a register
// load would also wait for every trajectory store before it).
__device__ __forceinline__ float2 lead_row(const Ext &x, int k, int S) {
    const int kk = k + (int)(threadIdx.x & 63);
    return kk <= S ? x.lead[kk] : make_float2(0.0f, 0.0f);
}

// The backward reads and writes the boundary rows through raw buffer
// resources: an absent row has zero records, so its loads return 0 and its
// stores are dropped without a memory access.  Every step then issues the
// same loads and stores, and the compiler can count the outstanding memory
// operations exactly instead of waiting for all of them.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Cache policy of the streams touched once: non-temporal (the `nt` bit of
// the gfx950 buffer instructions) for the forward's trajectory stores and the
// backward's per-step upstream loads (targets, dense upstream gradients);
// the checkpoints, written by the forward and read once by the backward, are
// non-temporal too.  Streaming them keeps L2 for the parameters and the
// exchange: on the 2M-vehicle workload, forward + backward 1.128 -> 1.098 ms
// with the trajectory stores, -> 1.070 ms with the upstream loads and ->
// 1.060 ms with the checkpoints (same-box A/Bs).
constexpr int kStreamNT = 2;

struct ExtRs {
    __amdgpu_buffer_rsrc_t lead, lead_adj, tail_adj;
    bool has_lead;
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const float2 *p, int n) {
    const char *c = reinterpret_cast<const char *>(reinterpret_cast<uintptr_t>(p));
    return __builtin_amdgcn_make_buffer_rsrc((void *)c, (short)0, p ? n * 8 : 0, 0x00020000);
}

__device__ __forceinline__ ExtRs ext_rsrc(const Ext &x, int S) {
    ExtRs r;
    r.lead = row_rsrc(x.lead, S + 1);
    r.lead_adj = row_rsrc(x.lead_adj, S);
    r.tail_adj = row_rsrc(x.tail_adj, S);
    r.has_lead = x.lead != nullptr;
    return r;
}

// Row entry k (k < 0 reads as 0; rows hold at most (2^27 + 1) entries of 8 B,
// so the offset 0x7ffffff0 is always outside them).
__device__ __forceinline__ float2 row_load(__amdgpu_buffer_rsrc_t rs, int k) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, k >= 0 ? k * 8 : 0x7ffffff0, 0, 0);
    return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}

// Thread 0 writes row entry k; every other lane's store falls outside the row.
__device__ __forceinline__ void row_store_t0(__amdgpu_buffer_rsrc_t rs, int k, float2 v) {
    const u32x2 d = {__float_as_uint(v.x), __float_as_uint(v.y)};
    __builtin_amdgcn_raw_buffer_store_b64(d, rs, threadIdx.x == 0 ? k * 8 : 0x7ffffff0, 0, 0);
}

// Leader states of thread 0 streamed one step ahead: `next` holds step k when
// step k starts; the step fetches k + 1 and keeps the value it used in `used`.
struct LeadPipe {
    float2 next, used;
};

__device__ __forceinline__ void lead_pipe_step(const ExtRs &xr, LeadPipe &lp, int k, float2 &L) {
    lp.used = lp.next;
    lp.next = row_load(xr.lead, k + 1);
    if (threadIdx.x == 0 && xr.has_lead) L = lp.used;
}

// CH: bundles may hold lane pieces (see k_backward).
// ER: both trajectory rows (displacements and speeds) are written, with the
// bundle-edge waves storing through the cache (see below); a separate
// instantiation, since the extra control flow costs the one-row forward 6-8 %
// even when it is not taken.
template <int MODE, int R, int NT, bool CH, bool ER>
__device__ __forceinline__ void forward_body(const SimArgs &A, float2 (*lead_buf)[64]) {
    __shared__ float2 sbuf[2][NT];
    __shared__ uint64_t dred[2][NT / 64];  // per-wave diagnostic counts
    const int t = threadIdx.x;
    const int tl = lead_thread(t);
    const int64_t N = A.n;
    const int S = A.n_steps;
    for (int bidx = blockIdx.x; bidx < A.n_bundles; bidx += gridDim.x) {
        Veh q[R];
        load_vehicles<R>(A, (int64_t)bidx * (NT * R) + t * R, q);
        const Ext x = ext_rows<CH>(A, bidx);
        float d[R], v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            d[r] = 0.0f;
            v[r] = q[r].g >= 0 ? A.v_init[q[r].g] : 0.0f;
            if (q[r].g >= 0) {
                if (A.traj_d) A.traj_d[q[r].g] = 0.0f;
                if (A.traj_v) A.traj_v[q[r].g] = v[r];
                if (A.ckpt) {
                    A.ckpt[q[r].g] = 0.0f;
                    A.ckpt[N + q[r].g] = v[r];
                }
            }
        }
        sbuf[0][t] = make_float2(d[R - 1], v[R - 1]);
        float2 lead_next = make_float2(0.0f, 0.0f);  // wave 0: the next 64-step chunk
        if constexpr (CH) {
            if (x.tail && t == NT - 1) x.tail[0] = make_float2(d[R - 1], v[R - 1]);
            if (x.lead && t < 64) {
                lead_buf[0][t] = lead_row(x, 0, S);
                lead_next = lead_row(x, 64, S);
            }
        }
        lds_barrier();
        // gap-floor diagnostics: each thread counts its evaluations ABOVE the
        // floor (one compare and one add on the vector unit, nothing that
        // makes the scalar unit wait for it); the floor count is the
        // complement, taken once after the last step.  A padding slot's
        // threshold is +inf, so it never counts as an evaluation.
        uint32_t n_ok = 0;
        float thr[R];
#pragma unroll
        for (int r = 0; r < R; ++r) thr[r] = q[r].g >= 0 ? A.gap_floor : INFINITY;
        int to_ckpt = A.K;  // steps until the next checkpoint
        // trajectory rows through raw buffer resources: the row address is
        // advanced by scalar adds, each lane stores at its loop-invariant byte
        // offset, and a padding slot's out-of-range offset drops its store
        const uint32_t NB = (uint32_t)(N * 4);
        int32_t voff[R];
#pragma unroll
        for (int r = 0; r < R; ++r)  // a padding slot's offset is the row size: always outside
            voff[r] = (int32_t)(q[r].g >= 0 ? (uint32_t)q[r].g * 4u : NB);
        // The first and last 128-byte lines of a bundle's part of a row are
        // shared with the neighbouring bundles whenever lanes do not end on a
        // 32-vehicle boundary.  Streamed (non-temporal) stores send those
        // partial lines to memory half-written, once from each side; with two
        // rows per step (displacements and speeds) that made the forward write
        // at 3.4 TB/s (0.46 ms on 2000 x 1000 vehicles, 0.32 ms with lanes of
        // 1024).  The waves holding a bundle's first or last vehicle therefore
        // store both rows through the cache when both are written: 0.39 ms.
        // (With one row, and in launches of few work-groups, where a step's
        // latency sets the time, the streamed stores are faster everywhere.)
        bool edge_cached = false;
        if constexpr (ER) {
            const int w = t >> 6;
            const int32_t first_g = __shfl(q[0].g, 0, 64);
            const int32_t last_g = __shfl(q[R - 1].g, 63, 64);
            bool edge = (w == 0);
            if (first_g >= 0) {
                // this wave holds the last real slot: its own last slot is
                // padding, it is the last wave, or the next wave starts with
                // padding (padding only ever follows the real slots)
                if (last_g < 0 || w == NT / 64 - 1)
                    edge = true;
                else if (A.slot_gidx[(int64_t)bidx * (NT * R) + (int64_t)(w + 1) * 64 * R] < 0)
                    edge = true;
            }
            edge_cached = __builtin_amdgcn_readfirstlane((int)edge) != 0;
        }
        const char *trow_d = reinterpret_cast<const char *>(A.traj_d);
        const char *trow_v = reinterpret_cast<const char *>(A.traj_v);
        // one step; P = k & 1 is a compile-time parity (the loop below runs
        // two steps per iteration: a barrier in the loop keeps the compiler
        // from unrolling it, and a run-time parity costs two address ops)
        auto fstep = [&](const int k, auto parity) {
            constexpr int P = decltype(parity)::value;
            float2 L = sbuf[P][tl];
            if constexpr (CH) {
                if (x.lead) {
                    const float2 X = lead_buf[(k >> 6) & 1][k & 63];
                    if (t == 0) L = X;
                    // last step of a chunk: stage the next one (read after this
                    // step's barrier) and fetch the one after
                    if ((k & 63) == 63 && t < 64) {
                        lead_buf[((k >> 6) + 1) & 1][t] = lead_next;
                        lead_next = lead_row(x, k + 65, S);
                    }
                }
            }
            float acc[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                // a lane head has g0 = +inf: any finite leader state gives a zero
                // interaction term
                float dh = r ? d[r - 1] : L.x;
                float vh = r ? v[r - 1] : L.y;
                // the lane model's gap (as in accel); a NaN gap counts as
                // floored, as the floor treats it
                const float gap = q[r].g0 + (dh - d[r]);
                n_ok += (gap > thr[r]) ? 1u : 0u;
                acc[r] = accel_gd<MODE>(q[r], v[r], gap, v[r] - vh, A.inv_dt, A.a_min,
                                        A.gap_floor);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) euler<MODE>(d[r], v[r], acc[r], A.dt);
            sbuf[P ^ 1][t] = make_float2(d[R - 1], v[R - 1]);
            if constexpr (CH)
                if (x.tail && t == NT - 1) x.tail[k + 1] = make_float2(d[R - 1], v[R - 1]);
            const bool ck = A.ckpt && (--to_ckpt == 0) && (k + 1 < S);
            if (to_ckpt == 0) to_ckpt = A.K;
            const int64_t crow = (int64_t)((k + 1) / A.K) * 2 * N;
            if (A.traj_d) {
                trow_d += NB;
                const __amdgpu_buffer_rsrc_t rs =
                    __builtin_amdgcn_make_buffer_rsrc((void *)trow_d, (short)0, (int)NB, 0x00020000);
if (edge_cached) {
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(d[r]), rs, voff[r], 0, 0);
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(d[r]), rs, voff[r], 0, kStreamNT);
                }
            }
            if (A.traj_v) {
                trow_v += NB;
                const __amdgpu_buffer_rsrc_t rs =
                    __builtin_amdgcn_make_buffer_rsrc((void *)trow_v, (short)0, (int)NB, 0x00020000);
if (edge_cached) {
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[r]), rs, voff[r], 0, 0);
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[r]), rs, voff[r], 0, kStreamNT);
                }
            }
            if (ck) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int32_t g = q[r].g;
                    if (g >= 0) {
                        __builtin_nontemporal_store(d[r], &A.ckpt[crow + g]);
                        __builtin_nontemporal_store(v[r], &A.ckpt[crow + N + g]);
                    }
                }
            }
            lds_barrier();
        };
        int k = 0;
        for (; k + 1 < S; k += 2) {
            fstep(k, std::integral_constant<int, 0>{});
            fstep(k + 1, std::integral_constant<int, 1>{});
        }
        if (k < S) fstep(k, std::integral_constant<int, 0>{});
        if (A.diag) {
            // A non-finite speed at any step makes every later displacement
            // non-finite (d' = d + dt v), so the final state shows whether the
            // vehicle's state was ever non-finite.
            uint64_t n_bad = 0;
#pragma unroll
            for (int r = 0; r < R; ++r)
                n_bad += (uint64_t)__builtin_popcountll(
                    __ballot(q[r].g >= 0 && !(isfinite(d[r]) && isfinite(v[r]))));
            uint32_t n_real = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) n_real += q[r].g >= 0 ? 1u : 0u;
            uint64_t n_floor = (uint64_t)(n_real * (uint32_t)S - n_ok);  // S < 2^27, R <= 4
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) n_floor += __shfl_down(n_floor, off, 64);
            if ((t & 63) == 0) {
                dred[0][t >> 6] = n_floor;
                dred[1][t >> 6] = n_bad;
            }
            lds_barrier();
            if (t == 0) {
                uint64_t s0 = 0, s1 = 0;
                for (int w = 0; w < NT / 64; ++w) {
                    s0 += dred[0][w];
                    s1 += dred[1][w];
                }
                A.diag[2 * (int64_t)bidx] = s0;
                A.diag[2 * (int64_t)bidx + 1] = s1;
            }
        }
    }
}


// Scalar registers: two 1024-thread work-groups share a compute unit only
// while a wave holds at most 80 SGPRs as the runtime counts them (96 halved
// the measured occupancy, 58 -> 31 resident waves per CU, and cost 55 % of
// the forward's time); the cap keeps the allocator below that.
template <int MODE, int R, int NT, bool ER>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_num_sgpr(72))) void k_forward(SimArgs A) {
    forward_body<MODE, R, NT, false, ER>(A, nullptr);
}

// Lane pieces (one vehicle per thread), with the register budget of 8 waves
// per SIMD: two 1024-thread work-groups per compute unit.
template <int MODE, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8))) void k_forward_pieces(
    SimArgs A) {
    __shared__ float2 lead_buf[2][64];
    forward_body<MODE, 1, NT, true, false>(A, lead_buf);
}

// Halo tiles: a lane too long to fill the chip with one work-group per lane
// is cut into tiles of threads - J owned vehicles, each run by its own
// work-group, and the steps into blocks of J run as successive launches.  A
// tile's forward slots are up to J vehicles ahead of the owned ones (the
// halo), then the owned vehicles, then padding; the first slot is flagged as
// a lane head.  Information travels one vehicle per step from leader to
// follower, so a halo vehicle without its true leader drifts from the true
// state from the front one vehicle per step, and after J steps the drift has
// not reached the owned vehicles.  The states at the block's first step are
// read from the trajectory rows, which the owners wrote in the previous
// launch; only owned vehicles write rows and count anomalies.  The per-vehicle
// arithmetic is the whole-lane forward's (accel_gd, euler), so the owned
// states equal it bit for bit.
template <int MODE, int NT>
__global__ __launch_bounds__(NT) void k_forward_tiled(SimArgs A) {
    __shared__ float2 sbuf[2][NT];
    __shared__ uint64_t dred[2][NT / 64];
    const int t = threadIdx.x;
    const int tl = lead_thread(t);
    const int64_t N = A.n;
    const int S = A.n_steps;
    const int k_lo = A.k_lo, k_hi = A.k_hi;
    const uint32_t NB = (uint32_t)(N * 4);
    for (int bidx = blockIdx.x; bidx < A.n_bundles; bidx += gridDim.x) {
        const int64_t slot = (int64_t)bidx * NT + t;
        Veh q[1];
        load_vehicles<1>(A, slot, q);
        const int32_t g = q[0].g;
        const bool own = g >= 0 && (A.slot_flags[slot] & SLOT_OWNED) != 0;
        float d = 0.0f, v = 0.0f;
        if (g >= 0) {
            if (k_lo == 0) {
                v = A.v_init[g];
            } else {
                d = A.traj_d[(int64_t)k_lo * N + g];
                v = A.traj_v[(int64_t)k_lo * N + g];
            }
        }
        if (k_lo == 0 && own) {
            A.traj_d[g] = 0.0f;
            A.traj_v[g] = v;
        }
        sbuf[0][t] = make_float2(d, v);
        lds_barrier();
        // evaluations above the gap floor (owned vehicles only; see forward_body)
        uint32_t n_ok = 0;
        const float thr = own ? A.gap_floor : INFINITY;
        // a slot that is not owned stores at the row size: outside the row
        const int32_t voff = (int32_t)(own ? (uint32_t)g * 4u : NB);
        const char *trow_d = reinterpret_cast<const char *>(A.traj_d) + (int64_t)k_lo * NB;
        const char *trow_v = reinterpret_cast<const char *>(A.traj_v) + (int64_t)k_lo * NB;
        auto step = [&](auto parity) {
            constexpr int P = decltype(parity)::value;
            const float2 L = sbuf[P][tl];
            const float gap = q[0].g0 + (L.x - d);
            n_ok += (gap > thr) ? 1u : 0u;
            const float acc = accel_gd<MODE>(q[0], v, gap, v - L.y, A.inv_dt, A.a_min, A.gap_floor);
            euler<MODE>(d, v, acc, A.dt);
            sbuf[P ^ 1][t] = make_float2(d, v);
            trow_d += NB;
            trow_v += NB;
            const __amdgpu_buffer_rsrc_t rd =
                __builtin_amdgcn_make_buffer_rsrc((void *)trow_d, (short)0, (int)NB, 0x00020000);
            const __amdgpu_buffer_rsrc_t rv =
                __builtin_amdgcn_make_buffer_rsrc((void *)trow_v, (short)0, (int)NB, 0x00020000);
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(d), rd, voff, 0, kStreamNT);
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rv, voff, 0, kStreamNT);
            lds_barrier();
        };
        int k = k_lo;
        for (; k + 1 < k_hi; k += 2) {
            step(std::integral_constant<int, 0>{});
            step(std::integral_constant<int, 1>{});
        }
        if (k < k_hi) step(std::integral_constant<int, 0>{});
        if (A.diag) {
            // floor counts add up over the launches; the non-finite count is
            // taken from the final state (see forward_body)
            uint64_t n_bad = (uint64_t)__builtin_popcountll(
                __ballot(own && !(isfinite(d) && isfinite(v))));
            uint64_t n_floor = (uint64_t)((own ? (uint32_t)(k_hi - k_lo) : 0u) - n_ok);
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) n_floor += __shfl_down(n_floor, off, 64);
            if ((t & 63) == 0) {
                dred[0][t >> 6] = n_floor;
                dred[1][t >> 6] = n_bad;
            }
            lds_barrier();
            if (t == 0) {
                uint64_t s0 = 0, s1 = 0;
                for (int w = 0; w < NT / 64; ++w) {
                    s0 += dred[0][w];
                    s1 += dred[1][w];
                }
                const uint64_t prev = k_lo == 0 ? 0 : A.diag[2 * (int64_t)bidx];
                A.diag[2 * (int64_t)bidx] = prev + s0;
                A.diag[2 * (int64_t)bidx + 1] = k_hi == S ? s1 : 0;
            }
        }
        __syncthreads();  // sbuf and dred are free before the next tile
    }
}

// ---------------------------------------------------------------- backward

// Raw upstream inputs of one (vehicle, step): dense dL/dd, dense dL/dv and the
// observed target.  Fetched one step ahead of their use so that the HBM
// latency overlaps a whole step of arithmetic.
struct Up {
    float gd, gv, tg;
};

// Walks the upstream inputs backwards one step at a time with a few scalar
// updates (no per-step multiply or division).  Loads go through buffer
// resources: an absent input, or the target row of an unobserved step, is a
// resource with zero records, whose loads return 0 without a memory access.
struct UpCursor {
    int64_t row;     // byte offset of step k's row in the dense inputs (k N 4)
    int64_t tg_row;  // byte offset of observation row `nobs` in the targets
    int k;           // step the cursor is on
    int nobs;        // largest observed step <= k, or INT_MIN if none is left
};

__device__ __forceinline__ void cursor_init(const SimArgs &A, int k, UpCursor &c) {
    const int64_t NB = A.n * 4;
    c.k = k;
    c.row = (int64_t)k * NB;
    c.nobs = INT_MIN;
    c.tg_row = 0;
    if (A.target && A.n_obs > 0 && k >= A.obs_first) {
        const int jq = min((k - A.obs_first) / A.obs_stride, A.n_obs - 1);
        c.nobs = A.obs_first + jq * A.obs_stride;
        c.tg_row = (int64_t)jq * NB;
    }
}

__device__ __forceinline__ bool cursor_obs(const UpCursor &c) { return c.k == c.nobs; }

__device__ __forceinline__ void cursor_dec(const SimArgs &A, UpCursor &c) {
    const int64_t NB = A.n * 4;
    if (c.k == c.nobs) {
        // leaving an observed step: the previous observation is a stride lower
        const int prev = c.nobs - A.obs_stride;
        c.nobs = prev >= A.obs_first ? prev : INT_MIN;
        c.tg_row -= NB;
    }
    c.k -= 1;
    c.row -= NB;
}

__device__ __forceinline__ float load_rec(const float *base, int64_t row, uint32_t bytes, int off) {
    // dword 3 of a raw (unswizzled, stride 0) buffer resource on gfx9; the
    // address is formed as an integer (the base may be null when bytes = 0)
    const char *p = reinterpret_cast<const char *>(reinterpret_cast<uintptr_t>(base) + row);
    __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, (int)bytes, 0x00020000);
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, kStreamNT));
}

// Loads of the cursor's step (padding slots read vehicle 0's word).  DN: the
// dense upstream inputs may be present; without them only the target is read.
// `live` = false (the cursor has passed step 0) reads nothing and gives zeros.
template <int R, bool DN>
__device__ __forceinline__ void fetch_up(const SimArgs &A, const UpCursor &c, const Veh (&q)[R],
                                         bool live, Up (&u)[R]) {
    // an absent input keeps its (null) base: with zero records the resource's
    // address is never used
    const uint32_t NB = live ? (uint32_t)(A.n * 4) : 0u;
    const uint32_t bgd = A.gd ? NB : 0u, bgv = A.gv ? NB : 0u;
    const uint32_t btg = cursor_obs(c) ? NB : 0u;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int off = (q[r].g > 0 ? q[r].g : 0) * 4;
        if constexpr (DN) {
            u[r].gd = load_rec(A.gd, c.row, bgd, off);
            u[r].gv = load_rec(A.gv, c.row, bgv, off);
        } else {
            u[r].gd = 0.0f;
            u[r].gv = 0.0f;
        }
        u[r].tg = load_rec(A.target, c.tg_row, btg, off);
    }
}

// fetch_up with explicit per-vehicle byte offsets (an offset beyond the row
// reads 0).
template <int R, bool DN>
__device__ __forceinline__ void fetch_up_at(const SimArgs &A, const UpCursor &c,
                                            const int (&off)[R], bool live, Up (&u)[R]) {
    const uint32_t NB = live ? (uint32_t)(A.n * 4) : 0u;
    const uint32_t bgd = A.gd ? NB : 0u, bgv = A.gv ? NB : 0u;
    const uint32_t btg = cursor_obs(c) ? NB : 0u;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if constexpr (DN) {
            u[r].gd = load_rec(A.gd, c.row, bgd, off[r]);
            u[r].gv = load_rec(A.gv, c.row, bgv, off[r]);
        } else {
            u[r].gd = 0.0f;
            u[r].gv = 0.0f;
        }
        u[r].tg = load_rec(A.target, c.tg_row, btg, off[r]);
    }
}

// Fused loss at one step: returns 2 (p - target) / |O| and adds the squared
// residual to `lossf`; 0 when the step is not observed.  p0 = p0h + p0l is
// split into two floats, and the residual is formed as ((p0h - target) + d)
// + p0l: the first difference cancels exactly when p0h and the target are
// within a factor of two, so the FP32 residual carries an error of about one
// unit in its own last place rather than in the position's.
__device__ __forceinline__ float mse_up(bool observed, bool valid, const Up &u, float d, float p0h,
                                        float p0l, float two_inv, float &lossf) {
    float s = 0.0f;
    if (observed) {
        float r = ((p0h - u.tg) + d) + p0l;
        r = valid ? r : 0.0f;
        lossf = fmaf(r, r, lossf);
        s = r * two_inv;
    }
    return s;
}

// One simulation step (step k) of all vehicles of the bundle (leader of the
// first vehicle from LDS or the boundary buffer, the others from registers),
// publishing the new state of the last vehicle into LDS buffer `nb` and ending
// on a barrier.
template <int MODE, int R, int NT, bool CH>
__device__ __forceinline__ void bundle_step(const SimArgs &A, const Veh (&q)[R], float (&d)[R],
                                            float (&v)[R], float2 (*sbuf)[NT], int cb, int nb,
                                            const ExtRs &xr, LeadPipe &lp, int k) {
    const int t = threadIdx.x;
    float2 L = sbuf[cb][lead_thread(t)];
    if constexpr (CH) lead_pipe_step(xr, lp, k, L);
    float acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float dh = r ? d[r - 1] : L.x;
        float vh = r ? v[r - 1] : L.y;
        acc[r] = accel<MODE>(q[r], d[r], v[r], dh, vh, A.inv_dt, A.a_min, A.gap_floor);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) euler<MODE>(d[r], v[r], acc[r], A.dt);
    sbuf[nb][t] = make_float2(d[R - 1], v[R - 1]);
    lds_barrier();
}

// Backward pass.  The forward stored a checkpoint every A.K steps; each
// checkpoint block is swept from its last KB-step sub-block to its first: the
// sub-block's start state is re-advanced from the checkpoint, its KB states are
// recomputed into registers, and the adjoint walks them backwards.  KB is a
// compile-time size (register arrays), A.K a multiple of it.
//
// ST (stash): when a block has exactly two sub-blocks, the re-advance to the
// upper one passes through every state of the lower one; they are kept in LDS
// (KB x NT*R float2) and the lower sub-block's reverse sweep reads them there
// instead of recomputing them, so each state of the block is computed once.
//
// DN: a dense upstream gradient (dL/dd or dL/dv) may be given; without it the
// kernel reads only the observed targets.
//
// CH: bundles may hold pieces of lanes longer than a bundle (boundary rows);
// without it that code is compiled out, keeping the register budget of the
// whole-lane kernels.
template <int MODE, int R, int NT, int KB, bool ST, bool DN, bool CH>
__global__ __launch_bounds__(NT) void k_backward(SimArgs A) {
    __shared__ float2 sbuf[2][NT];
    __shared__ float2 cbuf[2][NT];
    __shared__ float2 stash[ST ? KB : 1][ST ? NT * R : 1];
    // the final loss reduction reuses cbuf (after a barrier)
    double *red = reinterpret_cast<double *>(&cbuf[0][0]);
    static_assert((NT / 64 + 1) * sizeof(double) <= sizeof(cbuf), "reduction scratch");
    const int t = threadIdx.x;
    const int tl = lead_thread(t);             // leader's exchange slot
    const int tf = follow_thread<NT>(t);       // follower's contribution slot
    const int tlv = t > 0 ? t * R - 1 : 0;     // leader vehicle's stash slot
    const int64_t N = A.n;
    const int S = A.n_steps;
    const int K = A.K;
    const float dt = A.dt;
    const float two_inv = (float)A.two_inv_count;
    const int nblk = (S + K - 1) / K;
    for (int bidx = blockIdx.x; bidx < A.n_bundles; bidx += gridDim.x) {
        Veh q[R];
        load_vehicles<R>(A, (int64_t)bidx * (NT * R) + t * R, q);
        ExtRs xr{};
        if constexpr (CH) xr = ext_rsrc(ext_rows<CH>(A, bidx), S);
        LeadPipe lp{};
        float p0h[R], p0l[R];  // p0 = p0h + p0l
        float ld[R], lv[R];
        // dL/dp0: the gap terms plus the fused loss's direct term (p = p0 + d);
        // a dense upstream dL/dd acts at fixed p0 and reaches p0 only via gaps
        float gp0[R];
        double gacc[5][R];
        // squared residuals: FP32 per vehicle within a checkpoint block (the same
        // grouping for every launch shape), FP64 across blocks and vehicles
        double loss = 0.0;
        float lossf[R];
#pragma unroll
        for (int r = 0; r < R; ++r) lossf[r] = 0.0f;
        // upstream of the last step (the seed), and prefetch of step S-1
        // (two steps ahead: nxt = step k-1, nxt2 = step k-2 while step k is swept)
        Up seed[R], nxt[R], nxt2[R];
        UpCursor cur_k;
        cursor_init(A, S, cur_k);
        fetch_up<R, DN>(A, cur_k, q, true, seed);
        const bool obs_S = cursor_obs(cur_k);
        cursor_dec(A, cur_k);
        fetch_up<R, DN>(A, cur_k, q, S > 0, nxt);
        bool obs_nxt = S > 0 && cursor_obs(cur_k);
        cursor_dec(A, cur_k);
        fetch_up<R, DN>(A, cur_k, q, S > 1, nxt2);
        bool obs_nxt2 = S > 1 && cursor_obs(cur_k);
        // checkpoint of the last block
        float ckd[R], ckv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t gl = q[r].g > 0 ? q[r].g : 0;
            const int64_t crow = (int64_t)(nblk > 0 ? nblk - 1 : 0) * 2 * N;
            const double p0 = q[r].g >= 0 ? A.p0[gl] : 0.0;
            p0h[r] = (float)p0;
            p0l[r] = (float)(p0 - (double)p0h[r]);
            ckd[r] = nblk > 0 ? __builtin_nontemporal_load(&A.ckpt[crow + gl]) : 0.0f;
            ckv[r] = nblk > 0 ? __builtin_nontemporal_load(&A.ckpt[crow + N + gl]) : 0.0f;
            ld[r] = 0.0f;
            lv[r] = 0.0f;
            gp0[r] = 0.0f;
#pragma unroll
            for (int j = 0; j < 5; ++j) gacc[j][r] = 0.0;
        }
        if (S == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                gp0[r] = mse_up(obs_S, q[r].g >= 0, seed[r], 0.0f, p0h[r], p0l[r], two_inv, lossf[r]);
                ld[r] = seed[r].gd + gp0[r];
                lv[r] = seed[r].gv;
            }
        }
        for (int blk = nblk - 1; blk >= 0; --blk) {
            const int k0 = blk * K;
            const int len = min(K, S - k0);
            const int nsub = (len + KB - 1) / KB;
            // this block's checkpoint, kept for re-advancing to every sub-block
            float c0d[R], c0v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                c0d[r] = q[r].g >= 0 ? ckd[r] : 0.0f;
                c0v[r] = q[r].g >= 0 ? ckv[r] : 0.0f;
            }
            float gs[5][R];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int j = 0; j < 5; ++j) gs[j][r] = 0.0f;
            for (int sb = nsub - 1; sb >= 0; --sb) {
                const int ks = k0 + sb * KB;
                const int slen = min(KB, len - sb * KB);
                const bool stash_fill = ST && nsub == 2 && sb == 1;
                const bool stash_use = ST && nsub == 2 && sb == 0;
                float hd[KB][R], hv[KB][R];
                if (!stash_use) {
                    float d[R], v[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        d[r] = c0d[r];
                        v[r] = c0v[r];
                    }
                    if (stash_fill) {
                        // advance through the lower sub-block, keeping its states
#pragma unroll
                        for (int r = 0; r < R; ++r) stash[0][t * R + r] = make_float2(d[r], v[r]);
                        if constexpr (CH) lp.next = row_load(xr.lead, k0);
                        lds_barrier();
                        for (int j = 0; j < KB; ++j) {
                            float2 L = stash[j][tlv];
                            if constexpr (CH) lead_pipe_step(xr, lp, k0 + j, L);
                            float acc[R];
#pragma unroll
                            for (int r = 0; r < R; ++r) {
                                const float dh = r ? d[r - 1] : L.x;
                                const float vh = r ? v[r - 1] : L.y;
                                acc[r] = accel<MODE>(q[r], d[r], v[r], dh, vh, A.inv_dt, A.a_min,
                                                     A.gap_floor);
                            }
#pragma unroll
                            for (int r = 0; r < R; ++r) euler<MODE>(d[r], v[r], acc[r], dt);
                            if (j + 1 < KB) {
#pragma unroll
                                for (int r = 0; r < R; ++r)
                                    stash[j + 1][t * R + r] = make_float2(d[r], v[r]);
                            } else {
                                sbuf[0][t] = make_float2(d[R - 1], v[R - 1]);
                            }
                            lds_barrier();
                        }
                    } else {
                        sbuf[0][t] = make_float2(d[R - 1], v[R - 1]);
                        if constexpr (CH) lp.next = row_load(xr.lead, k0);
                        lds_barrier();
                        // re-advance from the checkpoint to the sub-block start
                        for (int j = 0; j < sb * KB; ++j)
                            bundle_step<MODE, R, NT, CH>(A, q, d, v, sbuf, j & 1, (j + 1) & 1,
                                                         xr, lp, k0 + j);
                        if (sb > 0) {
                            // restart the LDS ping-pong at parity 0 (buffer (sb*KB)&1
                            // was written last and is not read again)
                            sbuf[0][t] = make_float2(d[R - 1], v[R - 1]);
                            lds_barrier();
                        }
                    }
                    // recompute the sub-block's states into registers
#pragma unroll
                    for (int j = 0; j < KB; ++j) {
                        if (j < slen) {
#pragma unroll
                            for (int r = 0; r < R; ++r) {
                                hd[j][r] = d[r];
                                hv[j][r] = v[r];
                            }
                            bundle_step<MODE, R, NT, CH>(A, q, d, v, sbuf, j & 1, (j + 1) & 1,
                                                         xr, lp, ks + j);
                        }
                    }
                    if (blk == nblk - 1 && sb == nsub - 1) {
                        // seed: upstream gradient at the last step S (d, v are now step S)
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const float um = mse_up(obs_S, q[r].g >= 0, seed[r], d[r], p0h[r],
                                                    p0l[r], two_inv, lossf[r]);
                            gp0[r] += um;
                            ld[r] += seed[r].gd + um;
                            lv[r] += seed[r].gv;
                        }
                    }
                }
                if (sb == 0) {
                    // prefetch the previous block's checkpoint (block 0 reloads itself)
                    const int64_t crow = (int64_t)(blk > 0 ? blk - 1 : 0) * 2 * N;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int32_t gl = q[r].g > 0 ? q[r].g : 0;
                        ckd[r] = __builtin_nontemporal_load(&A.ckpt[crow + gl]);
                        ckv[r] = __builtin_nontemporal_load(&A.ckpt[crow + N + gl]);
                    }
                }
                // reverse sweep over the sub-block; its states come from the
                // registers or, for a stashed sub-block, from LDS.  The leader
                // state of the next step is read right after the barrier, next
                // to the follower's contribution, so a step waits on one LDS
                // round trip; a stashed sub-block reads its states one step
                // ahead, before the barrier (the stash is read-only here).
                float2 Lc;      // leader state of the current step
                float2 own[R];  // stashed sub-block: own states of the current step
                if (stash_use) {
#pragma unroll
                    for (int r = 0; r < R; ++r) own[r] = stash[KB - 1][t * R + r];
                    Lc = stash[KB - 1][tlv];
                } else {
                    Lc = sbuf[(slen - 1) & 1][tl];
                }
                // boundary rows of the sweep, one step ahead: the leader state of
                // step k-1 and the next piece head's contribution at step k
                float2 Xl_n = make_float2(0.0f, 0.0f), Xf_n = make_float2(0.0f, 0.0f);
                if constexpr (CH) {
                    // the last recomputed step used the leader state of step
                    // ks + slen - 1; a stashed sub-block recomputed nothing
                    const float2 Xlast =
                        stash_use ? row_load(xr.lead, ks + slen - 1) : lp.used;
                    if (t == 0 && xr.has_lead) Lc = Xlast;
                    Xl_n = row_load(xr.lead, ks + slen - 2);
                    Xf_n = row_load(xr.tail_adj, ks + slen - 1);
                }
                // (one step; j is a compile-time index on the register path)
                auto rstep = [&](const int j, auto from_stash) {
                    constexpr bool FS = decltype(from_stash)::value;
                    const int k = ks + j;
                    Up cur[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        cur[r] = nxt[r];
                        nxt[r] = nxt2[r];
                    }
                    const bool obs_cur = obs_nxt;
                    obs_nxt = obs_nxt2;
                    // prefetch step k-2 (nothing is read past step 0)
                    cursor_dec(A, cur_k);
                    fetch_up<R, DN>(A, cur_k, q, k > 1, nxt2);
                    obs_nxt2 = k > 1 && cursor_obs(cur_k);
                    // boundary rows of this step: the leader state of step k-1
                    // and the next piece head's contribution at step k
                    float2 Xl = make_float2(0.0f, 0.0f), Xf = make_float2(0.0f, 0.0f);
                    if constexpr (CH) {
                        Xl = Xl_n;
                        Xf = Xf_n;
                        Xl_n = row_load(xr.lead, k - 2);
                        Xf_n = row_load(xr.tail_adj, k - 1);
                    }
                    float sd[R], sv[R];
                    const float2 Lk = Lc;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        if constexpr (FS) {
                            sd[r] = own[r].x;
                            sv[r] = own[r].y;
                        } else {
                            sd[r] = hd[j][r];
                            sv[r] = hv[j][r];
                        }
                    }
                    if constexpr (FS) {
                        // next step's states, read now so that the LDS latency
                        // overlaps this step's arithmetic
                        if (j > 0) {
#pragma unroll
                            for (int r = 0; r < R; ++r) own[r] = stash[j - 1][t * R + r];
                            Lc = stash[j - 1][tlv];
                            if constexpr (CH)
                                if (t == 0 && xr.has_lead) Lc = Xl;
                        }
                    }
                    Part P[R];
                    float mu[R], mw[R], mwAs[R], um[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const float dh = r ? sd[r - 1] : Lk.x;
                        const float vh = r ? sv[r - 1] : Lk.y;
                        partials<MODE>(q[r], sd[r], sv[r], dh, vh, dt, A.inv_dt, A.a_min,
                                       A.gap_floor, P[r]);
                        mu[r] = (MODE == 0) ? dt * lv[r] : P[r].gate * dt * lv[r];
                        mw[r] = mu[r] * P[r].w;
                        mwAs[r] = mw[r] * P[r].As;
                        um[r] = mse_up(obs_cur, q[r].g >= 0, cur[r], sd[r], p0h[r], p0l[r],
                                       two_inv, lossf[r]);
                    }
                    // contribution of my first vehicle to its leader (previous
                    // thread): (mu d a*/d d_h, mu d a*/d v_h).  A lane head
                    // contributes exactly 0 (its hg and As vanish), so a lane
                    // tail needs no mask.
                    const float2 mine = make_float2(mw[0] * P[0].hg, -mwAs[0] * P[0].vc);
                    cbuf[j & 1][t] = mine;
                    if constexpr (CH) row_store_t0(xr.lead_adj, k, mine);
                    if constexpr (!FS) {
                        if (j > 0)
                            sbuf[(j - 1) & 1][t] = make_float2(hd[j - 1][R - 1], hv[j - 1][R - 1]);
                    }
                    lds_barrier();
                    float2 F = cbuf[j & 1][tf];
                    // the last thread's follower is thread 0 (exactly zero for a
                    // lane head) unless a boundary gives the next piece's head
                    if constexpr (CH)
                        if (t == NT - 1) F = Xf;
                    if constexpr (!FS) {
                        if (j > 0) {
                            Lc = sbuf[(j - 1) & 1][tl];
                            if constexpr (CH)
                                if (t == 0 && xr.has_lead) Lc = Xl;
                        }
                    }
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        float fd, fv;  // gathered from the follower
                        if (r + 1 < R) {
                            fd = mw[r + 1] * P[r + 1].hg;
                            fv = -mwAs[r + 1] * P[r + 1].vc;
                        } else {
                            fd = F.x;
                            fv = F.y;
                        }
                        const float gterm = fmaf(-mw[r], P[r].hg, fd);  // gap terms
                        const float gu = gterm + um[r];
                        float nlv = fmaf(dt, ld[r], P[r].carry * lv[r]);
                        nlv = fmaf(mwAs[r], P[r].u1, nlv);
                        nlv = fmaf(-mw[r] * q[r].fa_v0, P[r].x3, nlv);
                        nlv += fv;
                        // sufficient statistics of the five parameter gradients
                        gs[0][r] = fmaf(mw[r], P[r].x4, gs[0][r]);      // v0 (times 4a/v0)
                        gs[1][r] = fmaf(mwAs[r], sv[r], gs[1][r]);      // T
                        gs[2][r] = fmaf(mw[r], P[r].rest, gs[2][r]);    // a, direct part
                        gs[3][r] = fmaf(mwAs[r], P[r].vdvc, gs[3][r]);  // a and b, through c
                        gs[4][r] += mwAs[r];                           // s0
                        gp0[r] += gu;
                        if constexpr (DN) {
                            ld[r] = (ld[r] + gu) + cur[r].gd;
                            lv[r] = nlv + cur[r].gv;
                        } else {
                            ld[r] += gu;
                            lv[r] = nlv;
                        }
                    }
                };
                auto sweep_registers = [&]() {
#pragma unroll
                    for (int j = KB - 1; j >= 0; --j)
                        if (j < slen) rstep(j, std::false_type{});
                };
                if constexpr (ST) {
                    if (stash_use) {
                        // a stashed sub-block is always full; its states are
                        // indexed at run time.  Two steps per iteration remove
                        // most loop-carried register copies; a full unroll spills
#pragma unroll 2
                        for (int j = KB - 1; j >= 0; --j) rstep(j, std::true_type{});
                    } else {
                        sweep_registers();
                    }
                } else {
                    sweep_registers();
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                gacc[0][r] += (double)q[r].fa_v0 * (double)gs[0][r];
                gacc[1][r] += (double)gs[1][r];
                gacc[2][r] += (double)gs[2][r] - (double)q[r].i2a * (double)gs[3][r];
                gacc[3][r] -= (double)q[r].i2b * (double)gs[3][r];
                gacc[4][r] += (double)gs[4][r];
                loss += (double)lossf[r];
                lossf[r] = 0.0f;
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) loss += (double)lossf[r];  // S = 0: the seed's residual
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int32_t g = q[r].g;
            if (g >= 0) {
#pragma unroll
                for (int p = 0; p < 5; ++p) A.g_prm[(int64_t)p * N + g] = gacc[p][r];
                A.g_p0[g] = (double)gp0[r];
                A.g_v0[g] = (double)lv[r];
            }
        }
        __syncthreads();  // every cbuf read is done before the reduction reuses it
        double tot = block_sum(loss, red);
        if (t == 0 && A.loss_part) A.loss_part[bidx] = tot;
    }
}

// ---------------------------------------------------------------- backward from stored states
//
// The adjoint of k_backward for a caller that kept the forward's whole
// trajectory, displacements and speeds of every step ([S+1][N] each): the
// states of a step are read from it instead of being recomputed from
// checkpoints, so a step costs the partials and the adjoint update only.  A
// vehicle's leader is the previous vehicle of its lane, one index lower, so
// its state comes from the same rows (the first vehicle of a thread reads it
// at index g - 1, the others take it from registers) and the only exchange
// left is the follower's contribution, one LDS round trip and one barrier per
// step.  Every operation is the one k_backward performs, in the same order,
// and the FP32 gradient statistics are flushed into FP64 at the same
// K-step block boundaries, so the results equal k_backward's bit for bit for
// the same K.  Whole lanes only (no lane pieces).
struct StRow {
    float d, v;
};

// States of one step (row byte offset `row`): own vehicles and the first
// vehicle's leader.  `live` = false reads nothing and gives zeros.
template <int R>
__device__ __forceinline__ void fetch_states(const SimArgs &A, int64_t row, bool live,
                                             const int (&off)[R], int offl, StRow (&o)[R],
                                             StRow &lead) {
    const uint32_t NB = live ? (uint32_t)(A.n * 4) : 0u;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        o[r].d = load_rec(A.traj_d, row, NB, off[r]);
        o[r].v = load_rec(A.traj_v, row, NB, off[r]);
    }
    lead.d = load_rec(A.traj_d, row, NB, offl);
    lead.v = load_rec(A.traj_v, row, NB, offl);
}

//
// TL: a halo-tile launch (one vehicle per thread): it runs steps [k_lo, k_hi)
// of a tile whose slots are the owned vehicles followed by up to k_hi - k_lo
// halo followers.  The adjoint flows from follower to leader one vehicle per
// step; the tile's last vehicle lacks its follower's contribution, so the
// halo's adjoints go wrong from the back one vehicle per step, and after at
// most k_hi - k_lo steps the owned ones are still exact.  Every vehicle starts
// from the adjoint its owner carried out of the previous launch; only owned
// vehicles write results.  The arithmetic is the whole-lane kernel's.
template <int MODE, int R, int NT, bool DN, bool TL = false>
__global__ __launch_bounds__(NT) void k_backward_stored(SimArgs A) {
    static_assert(!TL || R == 1, "tiles hold one vehicle per thread");
    // one exchange buffer per ring slot: consecutive steps use different ones,
    // at addresses fixed at compile time
    __shared__ float2 cbuf[3][NT];
    double *red = reinterpret_cast<double *>(&cbuf[0][0]);
    static_assert((NT / 64 + 1) * sizeof(double) <= sizeof(cbuf), "reduction scratch");
    const int t = threadIdx.x;
    const int tf = follow_thread<NT>(t);
    const int64_t N = A.n;
    const int64_t NB = N * 4;
    const int S = A.n_steps;
    const int K = A.K;
    const float dt = A.dt;
    const float two_inv = (float)A.two_inv_count;
    // the launch's steps: all of them, or one block of a tile launch
    const int k_hi = TL ? A.k_hi : S;
    const int k_lo = TL ? A.k_lo : 0;
    const bool top = !TL || k_hi == S;
    for (int bidx = blockIdx.x; bidx < A.n_bundles; bidx += gridDim.x) {
        Veh q[R];
        load_vehicles<R>(A, (int64_t)bidx * (NT * R) + t * R, q);
        bool own = true;
        if constexpr (TL) own = (A.slot_flags[(int64_t)bidx * NT + t] & SLOT_OWNED) != 0;
        // byte offsets in a row: own vehicles and the first vehicle's leader
        // (a lane head, whose leader terms are exactly zero, reads its own
        // state).  A padding slot's offset lies beyond every row, so its
        // states, upstream inputs and target all read 0 and its residual is
        // exactly 0 without a select.
        int off[R];
#pragma unroll
        for (int r = 0; r < R; ++r) off[r] = q[r].g >= 0 ? q[r].g * 4 : INT_MAX - 3;
        const int offl = q[0].head ? off[0] : (q[0].g - 1) * 4;
        float p0h[R], p0l[R], ld[R], lv[R], gp0[R], lossf[R];
        float gs[5][R];
        double gacc[5][R];
        double loss = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t gl = q[r].g > 0 ? q[r].g : 0;
            const double p0 = q[r].g >= 0 ? A.p0[gl] : 0.0;
            p0h[r] = (float)p0;
            p0l[r] = (float)(p0 - (double)p0h[r]);
            ld[r] = 0.0f;
            lv[r] = 0.0f;
            gp0[r] = 0.0f;
            lossf[r] = 0.0f;
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                gs[j][r] = 0.0f;
                gacc[j][r] = 0.0;
            }
        }
        if constexpr (TL) {
            // below the top block: the adjoints carried out of the previous
            // launch (a halo vehicle's from its owner), and the owned
            // vehicles' running sums
            const int32_t g = q[0].g;
            if (!top && g >= 0) {
                ld[0] = A.tc_in[g];
                lv[0] = A.tc_in[N + g];
                if (own) {
                    gp0[0] = A.t_gp0[g];
#pragma unroll
                    for (int j = 0; j < 5; ++j) gacc[j][0] = A.t_acc[(int64_t)j * N + g];
                    loss = A.t_acc[5 * N + g];
                }
            }
        }
        // Three-slot rings of upstream inputs and states, read two steps
        // ahead: the step on step k reads slot `us` and refills slot `fs`,
        // the one the previous step read, with step k - 2 (a slot is never
        // refilled while its old values are still in use, so no value is
        // copied between registers and no load waits on a newer one).
        Up seed[R], up[3][R];
        bool obs_up[3];
        StRow st[3][R], lt[3];
        UpCursor cur_k;
        cursor_init(A, k_hi, cur_k);
        if (top) fetch_up_at<R, DN>(A, cur_k, off, true, seed);
        const bool obs_S = cursor_obs(cur_k);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            cursor_dec(A, cur_k);
            fetch_up_at<R, DN>(A, cur_k, off, k_hi > i, up[i]);
            obs_up[i] = k_hi > i && cursor_obs(cur_k);
            fetch_states<R>(A, (int64_t)(k_hi - 1 - i) * NB, k_hi > i, off, offl, st[i], lt[i]);
        }
        // seed: upstream gradient at step S (at S = 0 the state is the
        // initial one, displacement 0)
        if (top) {
            StRow sS[R], lS;
            fetch_states<R>(A, (int64_t)S * NB, S > 0, off, offl, sS, lS);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float dS = S > 0 ? sS[r].d : 0.0f;
                const float um = mse_up(obs_S, true, seed[r], dS, p0h[r], p0l[r], two_inv,
                                        lossf[r]);
                gp0[r] += um;
                ld[r] += seed[r].gd + um;
                lv[r] += seed[r].gv;
            }
        }
        // first step of the current K-step block (its statistics are flushed
        // into FP64 after that step)
        int kflush = k_hi > 0 ? ((k_hi - 1) / K) * K : 0;
        auto step = [&](const int k, auto use_slot, auto fill_slot) {
            constexpr int us = decltype(use_slot)::value;
            constexpr int fs = decltype(fill_slot)::value;
            Up cur[R];
            float sd[R], sv[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cur[r] = up[us][r];
                sd[r] = st[us][r].d;
                sv[r] = st[us][r].v;
            }
            const bool obs_cur = obs_up[us];
            const float2 Lk = make_float2(lt[us].d, lt[us].v);
            // step k - 2 (nothing is read before step 0)
            cursor_dec(A, cur_k);
            fetch_up_at<R, DN>(A, cur_k, off, k > 1, up[fs]);
            obs_up[fs] = k > 1 && cursor_obs(cur_k);
            fetch_states<R>(A, (int64_t)(k - 2) * NB, k > 1, off, offl, st[fs], lt[fs]);
            Part P[R];
            float mu[R], mw[R], mwAs[R], um[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float dh = r ? sd[r - 1] : Lk.x;
                const float vh = r ? sv[r - 1] : Lk.y;
                partials<MODE>(q[r], sd[r], sv[r], dh, vh, dt, A.inv_dt, A.a_min, A.gap_floor,
                               P[r]);
                mu[r] = (MODE == 0) ? dt * lv[r] : P[r].gate * dt * lv[r];
                mw[r] = mu[r] * P[r].w;
                mwAs[r] = mw[r] * P[r].As;
                um[r] = mse_up(obs_cur, true, cur[r], sd[r], p0h[r], p0l[r], two_inv, lossf[r]);
            }
            // my first vehicle's contribution to its leader, gathered by the
            // previous thread after the barrier (a lane head's is exactly 0)
            cbuf[us][t] = make_float2(mw[0] * P[0].hg, -mwAs[0] * P[0].vc);
            lds_barrier();
            const float2 F = cbuf[us][tf];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float fd, fv;
                if (r + 1 < R) {
                    fd = mw[r + 1] * P[r + 1].hg;
                    fv = -mwAs[r + 1] * P[r + 1].vc;
                } else {
                    fd = F.x;
                    fv = F.y;
                }
                const float gterm = fmaf(-mw[r], P[r].hg, fd);
                const float gu = gterm + um[r];
                float nlv = fmaf(dt, ld[r], P[r].carry * lv[r]);
                nlv = fmaf(mwAs[r], P[r].u1, nlv);
                nlv = fmaf(-mw[r] * q[r].fa_v0, P[r].x3, nlv);
                nlv += fv;
                gs[0][r] = fmaf(mw[r], P[r].x4, gs[0][r]);
                gs[1][r] = fmaf(mwAs[r], sv[r], gs[1][r]);
                gs[2][r] = fmaf(mw[r], P[r].rest, gs[2][r]);
                gs[3][r] = fmaf(mwAs[r], P[r].vdvc, gs[3][r]);
                gs[4][r] += mwAs[r];
                gp0[r] += gu;
                if constexpr (DN) {
                    ld[r] = (ld[r] + gu) + cur[r].gd;
                    lv[r] = nlv + cur[r].gv;
                } else {
                    ld[r] += gu;
                    lv[r] = nlv;
                }
            }
            if (k == kflush) {
                // FP32 statistics of the block into FP64
                kflush -= K;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    gacc[0][r] += (double)q[r].fa_v0 * (double)gs[0][r];
                    gacc[1][r] += (double)gs[1][r];
                    gacc[2][r] += (double)gs[2][r] - (double)q[r].i2a * (double)gs[3][r];
                    gacc[3][r] -= (double)q[r].i2b * (double)gs[3][r];
                    gacc[4][r] += (double)gs[4][r];
                    loss += (double)lossf[r];
                    lossf[r] = 0.0f;
#pragma unroll
                    for (int j = 0; j < 5; ++j) gs[j][r] = 0.0f;
                }
            }
        };
        using C0 = std::integral_constant<int, 0>;
        using C1 = std::integral_constant<int, 1>;
        using C2 = std::integral_constant<int, 2>;
        // slot 0 holds step k, slot 1 step k - 1 at the top of each iteration
        int k = k_hi - 1;
        for (; k >= k_lo + 2; k -= 3) {
            step(k, C0{}, C2{});
            step(k - 1, C1{}, C0{});
            step(k - 2, C2{}, C1{});
        }
        if (k == k_lo + 1) {
            step(k_lo + 1, C0{}, C2{});
            step(k_lo, C1{}, C0{});
        } else if (k == k_lo) {
            step(k_lo, C0{}, C2{});
        }
#pragma unroll
        for (int r = 0; r < R; ++r) loss += (double)lossf[r];  // S = 0: the seed's residual
        if constexpr (TL) {
            if (k_lo > 0) {
                // carried into the next launch: every owned vehicle's
                // adjoint and running sums (a tile's k_lo is a multiple of K,
                // so its FP32 statistics were just flushed)
                const int32_t g = q[0].g;
                if (g >= 0 && own) {
                    A.tc_out[g] = ld[0];
                    A.tc_out[N + g] = lv[0];
                    A.t_gp0[g] = gp0[0];
#pragma unroll
                    for (int j = 0; j < 5; ++j) A.t_acc[(int64_t)j * N + g] = gacc[j][0];
                    A.t_acc[5 * N + g] = loss;
                }
                __syncthreads();  // every cbuf read is done before the next tile writes it
                continue;
            }
            if (!own) loss = 0.0;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int32_t g = q[r].g;
            if (g >= 0 && own) {
#pragma unroll
                for (int p = 0; p < 5; ++p) A.g_prm[(int64_t)p * N + g] = gacc[p][r];
                A.g_p0[g] = (double)gp0[r];
                A.g_v0[g] = (double)lv[r];
            }
        }
        __syncthreads();  // every cbuf read is done before the reduction reuses it
        double tot = block_sum(loss, red);
        if (t == 0 && A.loss_part) A.loss_part[bidx] = tot;
    }
}

// ---------------------------------------------------------------- small kernels

__global__ __launch_bounds__(256) void k_loss_finalize(const double *part, int32_t n, double scale,
                                                       double *out) {
    __shared__ double red[5];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    double tot = block_sum(s, red);
    if (threadIdx.x == 0) *out = tot * scale;
}

// Sum of the per-bundle diagnostic counts [n][2]: integer sums, so the
// result does not depend on the order; 256 threads stride over the bundles,
// then a shared-memory tree.
__global__ __launch_bounds__(256) void k_diag_finalize(const uint64_t *part, int32_t n,
                                                       int64_t *out) {
    __shared__ uint64_t red[2][256];
    uint64_t s0 = 0, s1 = 0;
    for (int i = threadIdx.x; i < n; i += 256) {
        s0 += part[2 * (int64_t)i];
        s1 += part[2 * (int64_t)i + 1];
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = (int64_t)red[0][0];
        out[1] = (int64_t)red[1][0];
    }
}

__global__ __launch_bounds__(256) void k_fit_finalize(const double *part, int32_t n, double scale,
                                                      int32_t *step, double *hist,
                                                      int32_t hist_len) {
    __shared__ double red[5];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    double tot = block_sum(s, red);
    if (threadIdx.x == 0) {
        int32_t st = *step;
        hist[st < hist_len ? st : hist_len - 1] = tot * scale;
        *step = st + 1;
    }
}

// Adam (Kingma & Ba) on normalised parameters u in [0, 1], then projection
// onto the box and rewrite of the physical parameters lo + u (hi - lo).
__global__ __launch_bounds__(256) void k_adam(AdamArgs A) {
    const int64_t total = 5 * A.n;
    const int32_t t = *A.step;  // 1-based step number after the finalize kernel
    const float frac = fminf((float)(t - 1) / (float)A.lr_steps, 1.0f);
    const float lr = A.lr0 + (A.lr1 - A.lr0) * frac;
    const float bc1 = 1.0f - powf(A.beta1, (float)t);
    const float bc2 = 1.0f - powf(A.beta2, (float)t);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int p = (int)(i / A.n);
        float span = A.hi[p] - A.lo[p];
        // normalised: the moments follow dL/du = span dL/dtheta; raw units
        // (Sec. IV-A): they follow dL/dtheta and theta itself takes the step
        float g = A.raw ? (float)A.grad[i] : (float)(A.grad[i] * (double)span);
        float m = A.beta1 * A.m[i] + (1.0f - A.beta1) * g;
        float v = A.beta2 * A.v[i] + (1.0f - A.beta2) * g * g;
        A.m[i] = m;
        A.v[i] = v;
        float mh = m / bc1, vh = v / bc2;
        float step = lr * mh / (sqrtf(vh) + A.eps);
        if (A.raw) {
            float th = fminf(fmaxf(A.params[i] - step, A.lo[p]), A.hi[p]);
            A.params[i] = th;
            A.u[i] = (th - A.lo[p]) / span;
        } else {
            float u = fminf(fmaxf(A.u[i] - step, 0.0f), 1.0f);
            A.u[i] = u;
            A.params[i] = A.lo[p] + u * span;
        }
    }
}

// Fit initialisation: u = clamp((theta - lo) / (hi - lo), 0, 1), zero Adam
// moments, step counter 0, physical parameters rewritten from u.
__global__ __launch_bounds__(256) void k_fit_init(AdamArgs A, const float *init) {
    const int64_t total = 5 * A.n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int p = (int)(i / A.n);
        float span = A.hi[p] - A.lo[p];
        float u = fminf(fmaxf((init[i] - A.lo[p]) / span, 0.0f), 1.0f);
        A.u[i] = u;
        A.m[i] = 0.0f;
        A.v[i] = 0.0f;
        // raw units start from theta itself (projected onto the box)
        A.params[i] = A.raw ? fminf(fmaxf(init[i], A.lo[p]), A.hi[p]) : A.lo[p] + u * span;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *A.step_rw = 0;
}

__global__ __launch_bounds__(256) void k_params_from_u(AdamArgs A) {
    const int64_t total = 5 * A.n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int p = (int)(i / A.n);
        float u = fminf(fmaxf(A.u[i], 0.0f), 1.0f);
        A.u[i] = u;
        A.params[i] = A.lo[p] + u * (A.hi[p] - A.lo[p]);
    }
}

// Plain streaming copy (16-byte vectors, grid-stride): the measured HBM ceiling
// and the calibration reference of the hardware byte counters.
// Streaming copy (HBM ceiling and byte-counter calibration): each work-group
// moves chunks of 1024 16-byte words, four coalesced loads in flight per
// thread before its four stores, all non-temporal (the data is touched once).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                              int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * 1024;
    for (int64_t base = (int64_t)blockIdx.x * 1024; base < n16; base += stride) {
        u32x4 x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t i = base + j * 256 + threadIdx.x;
            if (i < n16) x[j] = __builtin_nontemporal_load(&src[i]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t i = base + j * 256 + threadIdx.x;
            if (i < n16) __builtin_nontemporal_store(x[j], &dst[i]);
        }
    }
}

// Observed positions from a displacement trajectory: out[j][i] =
// p0[i] + d[obs_first + j*obs_stride][i] (+ noise[j][i]), FP32.
__global__ __launch_bounds__(256) void k_observe(const float *traj_d, const double *p0,
                                                 const float *noise, int n_obs, int obs_first,
                                                 int obs_stride, int64_t N, float *out) {
    const int64_t total = (int64_t)n_obs * N;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = idx / N, i = idx - j * N;
        double p = p0[i] + (double)traj_d[(obs_first + j * obs_stride) * N + i];
        if (noise) p += (double)noise[idx];
        out[idx] = (float)p;
    }
}

// Sum over the vehicles of one lane and the observed steps of
// (p0 + d_k - target)^2, FP64, one work-group per lane, fixed order.
__global__ __launch_bounds__(256) void k_lane_loss(const float *traj_d, const double *p0,
                                                   const float *target, int n_obs, int obs_first,
                                                   int obs_stride, int64_t N,
                                                   const int32_t *lane_off, double *out) {
    __shared__ double red[5];
    const int l = blockIdx.x;
    const int lo = lane_off[l], hi = lane_off[l + 1];
    double s = 0.0;
    for (int i = lo + threadIdx.x; i < hi; i += blockDim.x)
        for (int j = 0; j < n_obs; ++j) {
            const int64_t k = obs_first + (int64_t)j * obs_stride;
            double r = p0[i] + (double)traj_d[k * N + i] - (double)target[(int64_t)j * N + i];
            s = fma(r, r, s);
        }
    double tot = block_sum(s, red);
    if (threadIdx.x == 0) out[l] = tot;
}

// out = lane's loss under A <= under B ? A : B, per vehicle, all 5 parameter blocks.
__global__ __launch_bounds__(256) void k_select_by_lane(const double *loss_a, const double *loss_b,
                                                        const int32_t *lane_of, const float *pa,
                                                        const float *pb, int64_t N, float *out,
                                                        int32_t *chose_a) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int l = lane_of[i];
        const bool a = loss_a[l] <= loss_b[l];
        for (int p = 0; p < 5; ++p) out[p * N + i] = a ? pa[p * N + i] : pb[p * N + i];
        if (chose_a) chose_a[i] = a ? 1 : 0;
    }
}

// Normalised parameters from a row-major [N][ld] source (first 5 columns),
// clamped to [0, 1], into the fit state (u, zero moments, step 0, params).
__global__ __launch_bounds__(256) void k_fit_init_u(AdamArgs A, const float *u_rows, int ld) {
    const int64_t total = 5 * A.n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(idx / A.n);
        const int64_t i = idx - (int64_t)p * A.n;
        const float u = fminf(fmaxf(u_rows[i * ld + p], 0.0f), 1.0f);
        A.u[idx] = u;
        A.m[idx] = 0.0f;
        A.v[idx] = 0.0f;
        A.params[idx] = A.lo[p] + u * (A.hi[p] - A.lo[p]);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *A.step_rw = 0;
}


}  // namespace

// ---------------------------------------------------------------- dispatch
//
// The file is compiled eleven times (IDM_PART = 0..10) so the backward
// instantiations of the two bound modes, with and without dense upstream
// gradients, with and without lane pieces, the backward from stored states
// (part 9) and the halo-tile kernels (part 10) build in parallel.
#ifndef IDM_PART
#define IDM_PART 0
#endif

#define IDM_FWD_CASE(M, R, NT)                                                \
    if (mode == M && per_thread == R && threads == NT)                        \
        return pieces ? (R == 1 ? (KernelFn)&k_forward_pieces<M, NT> : nullptr)  \
                      : (edge_cached ? (KernelFn)&k_forward<M, R, NT, true>       \
                                     : (KernelFn)&k_forward<M, R, NT, false>);
#define IDM_FWD_R(M, R) \
    IDM_FWD_CASE(M, R, 64) IDM_FWD_CASE(M, R, 128) IDM_FWD_CASE(M, R, 256) \
    IDM_FWD_CASE(M, R, 512) IDM_FWD_CASE(M, R, 1024)

#if IDM_PART == 0
KernelFn forward_kernel(int mode, int per_thread, int threads, bool pieces, bool edge_cached) {
    IDM_FWD_R(0, 1) IDM_FWD_R(0, 2) IDM_FWD_R(0, 4)
    IDM_FWD_R(1, 1) IDM_FWD_R(1, 2) IDM_FWD_R(1, 4)
    return nullptr;
}
#endif

#define IDM_BWD_CASE(M, R, NT, KK)                                            \
    if (mode == M && per_thread == R && threads == NT && KB == KK)            \
        return (KernelFn)&k_backward<M, R, NT, KK, false, IDM_DN, IDM_CH>;
// stash variants (checkpoint interval = two register blocks), for the shapes
// whose stash fits next to the exchange buffers in the 160 KB of LDS
#define IDM_BWD_ST(M, R, NT, KK)                                              \
    if (mode == M && per_thread == R && threads == NT && KB == KK && K == 2 * KK) \
        return (KernelFn)&k_backward<M, R, NT, KK, true, IDM_DN, IDM_CH>;
#define IDM_BWD_NT(M, R, KK)                                                  \
    IDM_BWD_CASE(M, R, 64, KK) IDM_BWD_CASE(M, R, 128, KK) IDM_BWD_CASE(M, R, 256, KK) \
    IDM_BWD_CASE(M, R, 512, KK) IDM_BWD_CASE(M, R, 1024, KK)
#define IDM_BWD_M(M)                                                          \
    IDM_BWD_ST(M, 1, 1024, 16) IDM_BWD_ST(M, 1, 512, 16) IDM_BWD_ST(M, 2, 512, 16) \
    IDM_BWD_ST(M, 4, 256, 8)                                                  \
    IDM_BWD_NT(M, 1, 8) IDM_BWD_NT(M, 1, 16) IDM_BWD_NT(M, 1, 32)             \
    IDM_BWD_NT(M, 2, 8) IDM_BWD_NT(M, 2, 16) IDM_BWD_NT(M, 2, 32)                \
    IDM_BWD_NT(M, 4, 4) IDM_BWD_NT(M, 4, 8)
// lane pieces: one vehicle per thread only
#define IDM_BWD_M_CH(M)                                                       \
    IDM_BWD_ST(M, 1, 1024, 16) IDM_BWD_ST(M, 1, 512, 16)                      \
    IDM_BWD_NT(M, 1, 8) IDM_BWD_NT(M, 1, 16) IDM_BWD_NT(M, 1, 32)

// parts 1-4: (softplus, clamp) x (targets only, dense upstream), whole lanes;
// parts 5-8: the same with lane pieces
#if IDM_PART >= 1 && IDM_PART <= 8
#define IDM_DN (IDM_PART == 3 || IDM_PART == 4 || IDM_PART == 7 || IDM_PART == 8)
#define IDM_CH (IDM_PART >= 5)
#define IDM_SP (IDM_PART == 1 || IDM_PART == 3 || IDM_PART == 5 || IDM_PART == 7)
#if IDM_PART == 1
KernelFn backward_kernel_sp_t(int mode, int per_thread, int threads, int KB, int K) {
#elif IDM_PART == 2
KernelFn backward_kernel_cl_t(int mode, int per_thread, int threads, int KB, int K) {
#elif IDM_PART == 3
KernelFn backward_kernel_sp_d(int mode, int per_thread, int threads, int KB, int K) {
#elif IDM_PART == 4
KernelFn backward_kernel_cl_d(int mode, int per_thread, int threads, int KB, int K) {
#elif IDM_PART == 5
KernelFn backward_kernel_sp_t_ch(int mode, int per_thread, int threads, int KB, int K) {
#elif IDM_PART == 6
KernelFn backward_kernel_cl_t_ch(int mode, int per_thread, int threads, int KB, int K) {
#elif IDM_PART == 7
KernelFn backward_kernel_sp_d_ch(int mode, int per_thread, int threads, int KB, int K) {
#else
KernelFn backward_kernel_cl_d_ch(int mode, int per_thread, int threads, int KB, int K) {
#endif
#if IDM_CH
    IDM_BWD_M_CH(IDM_SP ? 0 : 1)
#else
    IDM_BWD_M(IDM_SP ? 0 : 1)
#endif
    return nullptr;
}
#endif
#define IDM_BWS_CASE(M, R, NT)                                                 \
    if (mode == M && per_thread == R && threads == NT)                          \
        return dense ? (KernelFn)&k_backward_stored<M, R, NT, true>              \
                     : (KernelFn)&k_backward_stored<M, R, NT, false>;
#define IDM_BWS_R(M, R) \
    IDM_BWS_CASE(M, R, 64) IDM_BWS_CASE(M, R, 128) IDM_BWS_CASE(M, R, 256) \
    IDM_BWS_CASE(M, R, 512) IDM_BWS_CASE(M, R, 1024)
#if IDM_PART == 9
KernelFn backward_stored_kernel(int mode, int per_thread, int threads, bool dense) {
    IDM_BWS_R(0, 1) IDM_BWS_R(0, 2) IDM_BWS_R(0, 4)
    IDM_BWS_R(1, 1) IDM_BWS_R(1, 2) IDM_BWS_R(1, 4)
    return nullptr;
}
#endif

// part 10: the halo-tile kernels
#define IDM_TILE_CASE(M, NT)                                                   \
    if (mode == M && threads == NT) return (KernelFn)&k_forward_tiled<M, NT>;
#define IDM_TILE_BWD(M, NT)                                                    \
    if (mode == M && threads == NT)                                             \
        return dense ? (KernelFn)&k_backward_stored<M, 1, NT, true, true>        \
                     : (KernelFn)&k_backward_stored<M, 1, NT, false, true>;
#if IDM_PART == 10
// 576, 640 and 768 threads: a work-group only as wide as the tile needs
// (a 1000-vehicle lane in two tiles takes at most 564 slots at J = 128 and
// 628 at J = 256), since every wave of a work-group runs every step, padding
// or not
#define IDM_TILE_NT(X, M) X(M, 256) X(M, 512) X(M, 576) X(M, 640) X(M, 768) X(M, 1024)
KernelFn forward_tiled_kernel(int mode, int threads) {
    IDM_TILE_NT(IDM_TILE_CASE, 0) IDM_TILE_NT(IDM_TILE_CASE, 1)
    return nullptr;
}
KernelFn backward_tiled_kernel(int mode, int threads, bool dense) {
    IDM_TILE_NT(IDM_TILE_BWD, 0) IDM_TILE_NT(IDM_TILE_BWD, 1)
    return nullptr;
}
#endif

#if IDM_PART == 0
KernelFn backward_kernel_sp_t(int, int, int, int, int);
KernelFn backward_kernel_cl_t(int, int, int, int, int);
KernelFn backward_kernel_sp_d(int, int, int, int, int);
KernelFn backward_kernel_cl_d(int, int, int, int, int);
KernelFn backward_kernel_sp_t_ch(int, int, int, int, int);
KernelFn backward_kernel_cl_t_ch(int, int, int, int, int);
KernelFn backward_kernel_sp_d_ch(int, int, int, int, int);
KernelFn backward_kernel_cl_d_ch(int, int, int, int, int);
KernelFn backward_kernel(int mode, int per_thread, int threads, int KB, int K, bool dense,
                         bool pieces) {
    if (pieces) {
        if (dense)
            return mode == 0 ? backward_kernel_sp_d_ch(mode, per_thread, threads, KB, K)
                             : backward_kernel_cl_d_ch(mode, per_thread, threads, KB, K);
        return mode == 0 ? backward_kernel_sp_t_ch(mode, per_thread, threads, KB, K)
                         : backward_kernel_cl_t_ch(mode, per_thread, threads, KB, K);
    }
    if (dense)
        return mode == 0 ? backward_kernel_sp_d(mode, per_thread, threads, KB, K)
                         : backward_kernel_cl_d(mode, per_thread, threads, KB, K);
    return mode == 0 ? backward_kernel_sp_t(mode, per_thread, threads, KB, K)
                     : backward_kernel_cl_t(mode, per_thread, threads, KB, K);
}

hipError_t launch_sim(KernelFn fn, int grid, int threads, const SimArgs &a, hipStream_t s) {
    void *args[] = {(void *)&a};
    return hipLaunchKernel(fn, dim3(grid), dim3(threads), args, 0, s);
}

hipError_t launch_loss_finalize(const double *part, int32_t n_part, double scale, double *out,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_loss_finalize, dim3(1), dim3(256), 0, s, part, n_part, scale, out);
    return hipGetLastError();
}

hipError_t launch_diag_finalize(const uint64_t *part, int32_t n_part, int64_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_finalize, dim3(1), dim3(256), 0, s, part, n_part, out);
    return hipGetLastError();
}

hipError_t launch_fit_finalize(const double *part, int32_t n_part, double scale, int32_t *step,
                               double *hist, int32_t hist_len, hipStream_t s) {
    hipLaunchKernelGGL(k_fit_finalize, dim3(1), dim3(256), 0, s, part, n_part, scale, step, hist,
                       hist_len);
    return hipGetLastError();
}

static int elementwise_grid(int64_t total) {
    int64_t g = (total + 255) / 256;
    return (int)(g < 4096 ? (g < 1 ? 1 : g) : 4096);
}

hipError_t launch_copy(const void *src, void *dst, int64_t n16, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, s, (const u32x4 *)src, (u32x4 *)dst, n16);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(elementwise_grid(5 * a.n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fit_init(const AdamArgs &a, const float *init, hipStream_t s) {
    hipLaunchKernelGGL(k_fit_init, dim3(elementwise_grid(5 * a.n)), dim3(256), 0, s, a, init);
    return hipGetLastError();
}

hipError_t launch_observe(const float *traj_d, const double *p0, const float *noise, int n_obs,
                          int obs_first, int obs_stride, int64_t N, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_observe, dim3(elementwise_grid((int64_t)n_obs * N)), dim3(256), 0, s, traj_d,
                       p0, noise, n_obs, obs_first, obs_stride, N, out);
    return hipGetLastError();
}

hipError_t launch_lane_loss(const float *traj_d, const double *p0, const float *target, int n_obs,
                            int obs_first, int obs_stride, int64_t N, const int32_t *lane_off,
                            int n_lanes, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_lane_loss, dim3(n_lanes), dim3(256), 0, s, traj_d, p0, target, n_obs,
                       obs_first, obs_stride, N, lane_off, out);
    return hipGetLastError();
}

hipError_t launch_select_by_lane(const double *la, const double *lb, const int32_t *lane_of,
                                 const float *pa, const float *pb, int64_t N, float *out,
                                 int32_t *chose_a, hipStream_t s) {
    hipLaunchKernelGGL(k_select_by_lane, dim3(elementwise_grid(N)), dim3(256), 0, s, la, lb, lane_of,
                       pa, pb, N, out, chose_a);
    return hipGetLastError();
}

hipError_t launch_fit_init_u(const AdamArgs &a, const float *u_rows, int ld, hipStream_t s) {
    hipLaunchKernelGGL(k_fit_init_u, dim3(elementwise_grid(5 * a.n)), dim3(256), 0, s, a, u_rows, ld);
    return hipGetLastError();
}

hipError_t launch_params_from_u(const AdamArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_params_from_u, dim3(elementwise_grid(5 * a.n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

#endif  // IDM_PART == 0

}  // namespace idmx
