// HIP kernels of the ego-only trajectory reconstruction (arXiv 2412.16750,
// Sec. IV-A) for gfx950 (MI355X): every trajectory is one vehicle starting at
// p(0) = 0 whose leader is not simulated; the gap and speed difference to it
// at every step are free variables.  Forward, hand-derived adjoint of the
// summed absolute error, Adam with projection, nearest-step matching and the
// initial speed.  The IDM step is the lane kernels' (idm_device.h).
#include "idm_device.h"

#include <math.h>

namespace idmx {
namespace {

// ---------------------------------------------------------------- ego-only reconstruction
//
// One thread per trajectory (Sec. IV-A): the ego vehicle starts at p(0) = 0
// and its leader is not simulated; the gap and speed difference of every step
// are inputs ([S][N], step-major, so a wave's loads are coalesced).  No data
// is shared between threads, so these kernels have no LDS and no barrier.

constexpr int EGO_THREADS = 64;
constexpr int EGO_CHUNK = 8;  // steps whose free variables are loaded ahead

__device__ __forceinline__ void load_ego(const EgoArgs &A, int64_t i, Veh &q) {
    const float v0 = A.v0[i], a = A.a[i], b = A.b[i];
    q.inv_v0 = 1.0f / v0;
    q.T = A.T[i];
    q.a = a;
    q.s0 = A.s0[i];
    q.c = 0.5f / sqrtf(a * b);
    q.two_a = 2.0f * a;
    q.fa_v0 = 4.0f * a / v0;
    q.i2a = 0.5f / a;
    q.i2b = 0.5f / b;
    q.g0 = 0.0f;
    q.g = (int32_t)i;
    q.head = false;
}

template <int MODE>
__global__ __launch_bounds__(EGO_THREADS) void k_ego_forward(EgoArgs A) {
    const int64_t i = (int64_t)blockIdx.x * EGO_THREADS + threadIdx.x;
    if (i >= A.n) return;
    const int64_t N = A.n;
    const int S = A.n_steps;
    Veh q;
    load_ego(A, i, q);
    float d = 0.0f, v = A.v_init[i];
    if (A.traj_p) A.traj_p[i] = 0.0f;
    if (A.traj_v) A.traj_v[i] = v;
    if (A.ckpt) {
        A.ckpt[i] = 0.0f;
        A.ckpt[N + i] = v;
    }
    // free variables of the current and the next chunk of steps (indices
    // clamped into [0, S-1]; S = 0 reads nothing)
    float gc[EGO_CHUNK], dc[EGO_CHUNK];
#pragma unroll
    for (int u = 0; u < EGO_CHUNK; ++u) {
        const int64_t kk = min(u, S - 1);
        gc[u] = S > 0 ? A.gap[kk * N + i] : 0.0f;
        dc[u] = S > 0 ? A.dv[kk * N + i] : 0.0f;
    }
    int to_ckpt = A.K;
    for (int k0 = 0; k0 < S; k0 += EGO_CHUNK) {
        float gn[EGO_CHUNK], dn[EGO_CHUNK];
#pragma unroll
        for (int u = 0; u < EGO_CHUNK; ++u) {
            const int64_t kk = min(k0 + EGO_CHUNK + u, S - 1);
            gn[u] = A.gap[kk * N + i];
            dn[u] = A.dv[kk * N + i];
        }
#pragma unroll
        for (int u = 0; u < EGO_CHUNK; ++u) {
            const int k = k0 + u;
            if (k < S) {
                const float acc =
                    accel_gd<MODE>(q, v, gc[u], dc[u], A.inv_dt, A.a_min, A.gap_floor);
                const float vk = v;
                euler<MODE>(d, v, acc, A.dt);
                const int64_t row = (int64_t)(k + 1) * N + i;
                if (A.traj_p) A.traj_p[row] = d;
                if (A.traj_v) A.traj_v[row] = v;
                if (A.traj_a) A.traj_a[(int64_t)k * N + i] = MODE == 1 ? (v - vk) * A.inv_dt : acc;
                if (--to_ckpt == 0) {
                    to_ckpt = A.K;
                    if (A.ckpt && k + 1 < S) {
                        const int64_t c = (int64_t)((k + 1) / A.K) * 2 * N + i;
                        A.ckpt[c] = d;
                        A.ckpt[c + N] = v;
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < EGO_CHUNK; ++u) {
            gc[u] = gn[u];
            dc[u] = dn[u];
        }
    }
}

// The trajectory's next observations, walked from the last one backwards.
struct ObsRing {
    static constexpr int D = 4;
    int st[D];
    float pos[D];
    int j;     // index of the observation D places ahead of st[0]
    int lo;    // first observation of the trajectory
};

__device__ __forceinline__ void ring_fill(const EgoArgs &A, ObsRing &R, int lo, int hi) {
    R.lo = lo;
#pragma unroll
    for (int u = 0; u < ObsRing::D; ++u) {
        const int j = hi - 1 - u;
        R.st[u] = j >= lo ? A.obs_step[j] : -1;
        R.pos[u] = j >= lo ? A.obs_pos[j] : 0.0f;
    }
    R.j = hi - 1 - ObsRing::D;
}

// Upstream dL/dp at step k from the observations matched to k (summed
// absolute error: sign(p - obs), 0 at equality); their |p - obs| go to `loss`.
__device__ __forceinline__ float ring_take(const EgoArgs &A, ObsRing &R, int k, float p,
                                           double &loss) {
    float up = 0.0f;
    while (R.st[0] == k) {
        const float r = p - R.pos[0];
        up += (r > 0.0f ? 1.0f : 0.0f) - (r < 0.0f ? 1.0f : 0.0f);
        loss += (double)fabsf(r);
#pragma unroll
        for (int u = 0; u + 1 < ObsRing::D; ++u) {
            R.st[u] = R.st[u + 1];
            R.pos[u] = R.pos[u + 1];
        }
        const int j = R.j;
        R.st[ObsRing::D - 1] = j >= R.lo ? A.obs_step[j] : -1;
        R.pos[ObsRing::D - 1] = j >= R.lo ? A.obs_pos[j] : 0.0f;
        R.j = j - 1;
    }
    return up;
}

// Ego backward: checkpoint blocks of K = KB steps from the last; each block's
// states and free variables are recomputed into registers, then the adjoint
// walks them backwards.  Per step it writes dL/dG and dL/dD (non-temporal:
// read once, by the optimiser; the reconstruction fit step 1.118 -> 1.087 ms
// in a same-box A/B); the parameter gradients accumulate as the five
// sufficient statistics of the lane kernel.
template <int MODE, int KB>
__global__ __launch_bounds__(EGO_THREADS) void k_ego_backward(EgoArgs A) {
    const int64_t i = (int64_t)blockIdx.x * EGO_THREADS + threadIdx.x;
    if (i >= A.n) return;
    const int64_t N = A.n;
    const int S = A.n_steps;
    const float dt = A.dt;
    const int nblk = (S + KB - 1) / KB;
    Veh q;
    load_ego(A, i, q);
    ObsRing R;
    ring_fill(A, R, A.obs_off[i], A.obs_off[i + 1]);
    double loss = 0.0;
    double gacc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    float lp = 0.0f, lv = 0.0f;
    if (S == 0) lp = ring_take(A, R, 0, 0.0f, loss);
    for (int blk = nblk - 1; blk >= 0; --blk) {
        const int k0 = blk * KB;
        const int len = min(KB, S - k0);
        const int64_t c = (int64_t)blk * 2 * N + i;
        float d = A.ckpt[c], v = A.ckpt[c + N];
        float hd[KB], hv[KB], hg[KB], hq[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) {
            const int64_t kk = (int64_t)min(k0 + j, S - 1) * N + i;
            hg[j] = A.gap[kk];
            hq[j] = A.dv[kk];
        }
#pragma unroll
        for (int j = 0; j < KB; ++j) {
            if (j < len) {
                hd[j] = d;
                hv[j] = v;
                const float acc = accel_gd<MODE>(q, v, hg[j], hq[j], A.inv_dt, A.a_min, A.gap_floor);
                euler<MODE>(d, v, acc, dt);
            }
        }
        if (blk == nblk - 1) lp = ring_take(A, R, S, d, loss);  // seed: step S
        float gs[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int j = KB - 1; j >= 0; --j) {
            if (j < len) {
                const int k = k0 + j;
                Part P;
                partials_gd<MODE, true>(q, hv[j], hg[j], hq[j], dt, A.inv_dt, A.a_min,
                                        A.gap_floor, P);
                const float mu = (MODE == 0) ? dt * lv : P.gate * dt * lv;
                const float mw = mu * P.w;
                const float mwAs = mw * P.As;
                __builtin_nontemporal_store(mw * P.hg, &A.g_gap[(int64_t)k * N + i]);
                __builtin_nontemporal_store(mwAs * P.vc, &A.g_dv[(int64_t)k * N + i]);
                float nlv = fmaf(dt, lp, P.carry * lv);
                nlv = fmaf(mwAs, P.u1, nlv);
                nlv = fmaf(-mw * q.fa_v0, P.x3, nlv);
                gs[0] = fmaf(mw, P.x4, gs[0]);
                gs[1] = fmaf(mwAs, hv[j], gs[1]);
                gs[2] = fmaf(mw, P.rest, gs[2]);
                gs[3] = fmaf(mwAs, P.vdvc, gs[3]);
                gs[4] += mwAs;
                lp += ring_take(A, R, k, hd[j], loss);
                lv = nlv;
            }
        }
        gacc[0] += (double)q.fa_v0 * (double)gs[0];
        gacc[1] += (double)gs[1];
        gacc[2] += (double)gs[2] - (double)q.i2a * (double)gs[3];
        gacc[3] -= (double)q.i2b * (double)gs[3];
        gacc[4] += (double)gs[4];
    }
#pragma unroll
    for (int p = 0; p < 5; ++p) A.g_prm[(int64_t)p * N + i] = gacc[p];
    if (A.g_v0) A.g_v0[i] = (double)lv;
    A.loss_part[i] = loss;
}

// Adam (Kingma & Ba) on the physical parameters, projected onto their boxes,
// and on the unconstrained per-step gap and speed difference; learning rate
// linear from lr0 to lr1 over lr_steps.  The per-step gradients and the
// moments are touched once per fit step and dwarf the caches, so they stream
// non-temporally (the reconstruction fit step 1.17 -> 1.11 ms, the filtering
// one 1.38 -> 1.25 ms in a same-box A/B); the variables themselves, read again
// by the next forward, keep the default policy.
__global__ __launch_bounds__(256) void k_ego_adam(EgoAdamArgs A) {
    const int64_t n5 = 5 * A.n, total = n5 + 2 * A.sn;
    const int32_t t = *A.step;
    const float frac = fminf((float)(t - 1) / (float)A.lr_steps, 1.0f);
    const float lr = A.lr0 + (A.lr1 - A.lr0) * frac;
    const float bc1 = 1.0f - powf(A.beta1, (float)t);
    const float bc2 = 1.0f - powf(A.beta2, (float)t);
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        float x, g;
        if (idx < n5) {
            x = A.params[idx];
            g = (float)A.g_prm[idx];
        } else if (idx < n5 + A.sn) {
            x = A.gap[idx - n5];
            g = __builtin_nontemporal_load(&A.g_gap[idx - n5]);
        } else {
            x = A.dv[idx - n5 - A.sn];
            g = __builtin_nontemporal_load(&A.g_dv[idx - n5 - A.sn]);
        }
        const float m = A.beta1 * __builtin_nontemporal_load(&A.m[idx]) + (1.0f - A.beta1) * g;
        const float v = A.beta2 * __builtin_nontemporal_load(&A.v[idx]) + (1.0f - A.beta2) * g * g;
        __builtin_nontemporal_store(m, &A.m[idx]);
        __builtin_nontemporal_store(v, &A.v[idx]);
        x -= lr * (m / bc1) / (sqrtf(v / bc2) + A.eps);
        if (idx < n5) {
            const int p = (int)(idx / A.n);
            A.params[idx] = fminf(fmaxf(x, A.lo[p]), A.hi[p]);
        } else if (idx < n5 + A.sn) {
            A.gap[idx - n5] = x;
        } else {
            A.dv[idx - n5 - A.sn] = x;
        }
    }
}

// Initial values of the fit: parameters init5[p] for every trajectory, gap
// gap0 and speed difference dv0 at every step, zero moments, step 0.
__global__ __launch_bounds__(256) void k_ego_fit_init(EgoAdamArgs A, float i0, float i1, float i2,
                                                      float i3, float i4, float gap0, float dv0) {
    const int64_t n5 = 5 * A.n, total = n5 + 2 * A.sn;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        if (idx < n5) {
            const int p = (int)(idx / A.n);
            A.params[idx] = p == 0 ? i0 : p == 1 ? i1 : p == 2 ? i2 : p == 3 ? i3 : i4;
        } else if (idx < n5 + A.sn) {
            A.gap[idx - n5] = gap0;
        } else {
            A.dv[idx - n5 - A.sn] = dv0;
        }
        A.m[idx] = 0.0f;
        A.v[idx] = 0.0f;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *A.step_rw = 0;
}

// Nearest simulation step of each timestamp (Sec. IV-A), clamped to [0, S].
__global__ __launch_bounds__(256) void k_ego_match_steps(const double *t, int32_t m, double dt,
                                                         int32_t n_steps, int32_t *out) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m;
         j += (int64_t)gridDim.x * blockDim.x) {
        double k = rint(t[j] / dt);
        k = k < 0.0 ? 0.0 : (k > (double)n_steps ? (double)n_steps : k);
        out[j] = (int32_t)k;
    }
}

// Initial speed of each trajectory from its first two observations (Sec. V-B3):
// max((P_1 - P_0) / (T_1 - T_0), 0); 0 with fewer than two observations.
__global__ __launch_bounds__(256) void k_ego_initial_speed(const int32_t *off, const double *t,
                                                           const float *pos, int64_t n, float *v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int lo = off[i], hi = off[i + 1];
        float s = 0.0f;
        if (hi - lo >= 2) {
            const double dtj = t[lo + 1] - t[lo];
            if (dtj > 0.0) s = (float)(((double)pos[lo + 1] - (double)pos[lo]) / dtj);
        }
        v[i] = fmaxf(s, 0.0f);
    }
}

static int elementwise_grid(int64_t total) {
    int64_t g = (total + 255) / 256;
    return (int)(g < 4096 ? (g < 1 ? 1 : g) : 4096);
}

}  // namespace

hipError_t launch_ego_forward(int mode, const EgoArgs &a, hipStream_t s) {
    const dim3 grid((unsigned)((a.n + EGO_THREADS - 1) / EGO_THREADS));
    if (mode == 0)
        hipLaunchKernelGGL(k_ego_forward<0>, grid, dim3(EGO_THREADS), 0, s, a);
    else
        hipLaunchKernelGGL(k_ego_forward<1>, grid, dim3(EGO_THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ego_backward(int mode, const EgoArgs &a, hipStream_t s) {
    const dim3 grid((unsigned)((a.n + EGO_THREADS - 1) / EGO_THREADS)), blk(EGO_THREADS);
#define IDM_EGO_BWD(M, KK) \
    if (mode == M && a.K == KK) { hipLaunchKernelGGL((k_ego_backward<M, KK>), grid, blk, 0, s, a); return hipGetLastError(); }
    IDM_EGO_BWD(0, 8) IDM_EGO_BWD(0, 16) IDM_EGO_BWD(0, 32)
    IDM_EGO_BWD(1, 8) IDM_EGO_BWD(1, 16) IDM_EGO_BWD(1, 32)
#undef IDM_EGO_BWD
    return hipErrorInvalidValue;
}

hipError_t launch_ego_adam(const EgoAdamArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_ego_adam, dim3(elementwise_grid(5 * a.n + 2 * a.sn)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ego_fit_init(const EgoAdamArgs &a, const float *init5, float gap0, float dv0,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_ego_fit_init, dim3(elementwise_grid(5 * a.n + 2 * a.sn)), dim3(256), 0, s,
                       a, init5[0], init5[1], init5[2], init5[3], init5[4], gap0, dv0);
    return hipGetLastError();
}

hipError_t launch_ego_match_steps(const double *t, int32_t m, double dt, int32_t n_steps,
                                  int32_t *step_out, hipStream_t s) {
    hipLaunchKernelGGL(k_ego_match_steps, dim3(elementwise_grid(m)), dim3(256), 0, s, t, m, dt,
                       n_steps, step_out);
    return hipGetLastError();
}

hipError_t launch_ego_initial_speed(const int32_t *off, const double *t, const float *pos,
                                    int64_t n, float *v_out, hipStream_t s) {
    hipLaunchKernelGGL(k_ego_initial_speed, dim3(elementwise_grid(n)), dim3(256), 0, s, off, t, pos,
                       n, v_out);
    return hipGetLastError();
}

}  // namespace idmx
