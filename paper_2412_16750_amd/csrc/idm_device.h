// Device math shared by the lane kernels (idm_kernels.hip) and the ego-only
// reconstruction kernels (ego_kernels.hip): the IDM acceleration with the
// paper's bounds (Sec. III-A Eqs. 1-3, Sec. III-C), its local partial
// derivatives, the Euler step, the LDS-only barrier and a fixed-order
// work-group sum.  Everything is inline and internal to each translation unit.
#pragma once

#include "idm_internal.h"

#include <math.h>

namespace idmx {
namespace {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float log2_fast(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }

// softplus(x) = log(1 + e^x) = max(x, 0) + log(1 + e^-|x|)   (Sec. III-C)
__device__ __forceinline__ float softplus(float x) {
    float e = exp2_fast(-fabsf(x) * kLog2e);
    return fmaf(kLn2, log2_fast(1.0f + e), fmaxf(x, 0.0f));
}

// softplus(x) and its derivative, the logistic function.
__device__ __forceinline__ float softplus_d(float x, float &sig) {
    float e = exp2_fast(-fabsf(x) * kLog2e);
    float onep = 1.0f + e;
    float r = rcp_fast(onep);
    sig = x >= 0.0f ? r : e * r;
    return fmaf(kLn2, log2_fast(onep), fmaxf(x, 0.0f));
}

// Work-group barrier that orders only LDS traffic.  __syncthreads() also
// waits for every outstanding global store of the wave, which would stall each
// time step on the trajectory writes; nothing here reads another thread's
// global writes inside a launch, so only the LDS ("local") fence is needed.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// 1 / (1 + e^-x).  For x << 0 the exponential overflows to +inf and the
// reciprocal gives the limit 0; no NaN for any finite x.
__device__ __forceinline__ float logistic(float x) {
    return rcp_fast(1.0f + exp2_fast(-x * kLog2e));
}

// Per-vehicle constants, computed once per launch.
struct Veh {
    float inv_v0, T, a, s0;
    float c;      // 1 / (2 sqrt(a b))   (Eq. 1)
    float g0;     // initial gap to the leader (FP64 difference, rounded); +inf for a lane head
    float two_a;  // 2 a
    float fa_v0;  // 4 a / v0   (delta = 4)
    float i2a, i2b;  // 1 / (2a), 1 / (2b)
    int32_t g;    // global vehicle index, -1 for padding
    bool head;
};

// Acceleration entering the speed update: a* (SOFTPLUS) or ahat (CLAMP), for
// a bumper-to-bumper gap and speed difference v - v_h to the leader.
template <int MODE>
__device__ __forceinline__ float accel_gd(const Veh &q, float v, float gap, float dv,
                                          float inv_dt, float a_min, float gap_floor) {
    float x = v * q.inv_v0;
    float x2 = x * x;
    float sg = fmaxf(gap, gap_floor);
    float s_opt = fmaf(v * dv, q.c, fmaf(v, q.T, q.s0));  // Eq. 1
    float s = (MODE == 0) ? softplus(s_opt) : s_opt;  // Sec. III-C floor on s_opt
    float qq = s * rcp_fast(sg);
    float rest = 1.0f - fmaf(qq, qq, x2 * x2);          // Eq. 2, delta = 4: ahat = a rest
    if (MODE == 0) {
        // Sec. III-C: a* = a_lb + softplus(ahat - a_lb), a_lb = max(-v/dt, a_min),
        // carried as -a_lb = min(v/dt, -a_min)
        float mlb = fminf(v * inv_dt, -a_min);
        return softplus(fmaf(q.a, rest, mlb)) - mlb;
    }
    return q.a * rest;
}

// The lane model: gap = p_h - p - len_h = g0 + (d_h - d), dv = v - v_h
// (Sec. III-A).  A lane head has g0 = +inf, so its interaction term is
// exactly zero.
template <int MODE>
__device__ __forceinline__ float accel(const Veh &q, float d, float v, float dh, float vh,
                                       float inv_dt, float a_min, float gap_floor) {
    return accel_gd<MODE>(q, v, q.g0 + (dh - d), v - vh, inv_dt, a_min, gap_floor);
}

template <int MODE>
__device__ __forceinline__ void euler(float &d, float &v, float acc, float dt) {
    float dn = fmaf(dt, v, d);                        // Eq. 3, old speed
    float vn = fmaf(dt, acc, v);
    if (MODE == 1) vn = fmaxf(vn, 0.0f);
    d = dn;
    v = vn;
}

// Local partial derivatives at one (vehicle, step).  With ahat the IDM
// acceleration of Eq. 2, a* the bounded one that enters the speed update,
// gap = g0 + d_h - d and s_opt of Eq. 1:
//   d a*/d gap  = w hg
//   d a*/d v    = w (As (T + (dv + v) c) - (4a/v0) x^3) + (d a_lb/d v)(1 - w)
//   d a*/d v_h  = -w As v c
//   d a*/d v0   = w (4a/v0) x^4,   d a*/d T = w As v,   d a*/d s0 = w As,
//   d a*/d a    = w (rest - As v dv c / (2a)),   d a*/d b = -w As v dv c / (2b)
// with As = d ahat / d s_opt and rest = 1 - x^4 - (s*/gap)^2.
struct Part {
    float hg;      // d ahat / d gap (0 while the gap floor is active)
    float As;      // d ahat / d s_opt
    float u1;      // T + (dv + v) c  = d s_opt / d v
    float x3, x4;  // (v/v0)^3, (v/v0)^4
    float vc;      // v c
    float vdvc;    // v dv c
    float rest;    // 1 - x^4 - (s*/gap)^2
    float w;       // d a* / d ahat (1 in CLAMP mode)
    float gate;    // d v' / d (v + dt a*): 1, or the clamp indicator
    float carry;   // d v' / d v apart from the ahat terms: with the bound on
                   // a_lb = -v/dt its -1/dt (1 - w) cancels all but w of the
                   // Euler update's 1 (w then, 1 on a_min); the clamp
                   // indicator in CLAMP mode
};

// EGO: the speed difference is a free input (the ego-only reconstruction
// model), so d s_opt / d v = T + dv c instead of T + (dv + v) c.
template <int MODE, bool EGO = false>
__device__ __forceinline__ void partials_gd(const Veh &q, float v, float gap, float dv, float dt,
                                            float inv_dt, float a_min, float gap_floor, Part &P) {
    float x = v * q.inv_v0;
    float x2 = x * x;
    bool floored = !(gap > gap_floor);
    float sg = fmaxf(gap, gap_floor);  // = floored ? gap_floor : gap (a NaN gap too), as in accel_gd
    float inv_sg = rcp_fast(sg);
    float vdv = v * dv;
    float s_opt = fmaf(vdv, q.c, fmaf(v, q.T, q.s0));
    float sig_s = 1.0f, s = s_opt;
    if (MODE == 0) s = softplus_d(s_opt, sig_s);
    float qq = s * inv_sg;
    P.x4 = x2 * x2;
    P.rest = 1.0f - fmaf(qq, qq, P.x4);
    float tq = q.two_a * qq * inv_sg;                 // 2 a q / gap
    P.As = -tq * sig_s;
    P.hg = floored ? 0.0f : tq * qq;                  // 2 a q^2 / gap
    P.u1 = EGO ? fmaf(dv, q.c, q.T) : fmaf(dv + v, q.c, q.T);
    P.x3 = x2 * x;
    P.vc = v * q.c;
    P.vdvc = vdv * q.c;
    if (MODE == 0) {
        // a_lb = max(-v/dt, a_min) (tie -> a_min branch), entering as -a_lb
        float pv = v * inv_dt;
        bool on_v = pv < -a_min;
        float mlb = fminf(pv, -a_min);  // = on_v ? pv : -a_min, as in accel_gd
        P.w = logistic(fmaf(q.a, P.rest, mlb));       // ahat - a_lb
        P.gate = 1.0f;
        P.carry = on_v ? P.w : 1.0f;
    } else {
        float ahat = q.a * P.rest;
        P.w = 1.0f;
        P.gate = (fmaf(dt, ahat, v) > 0.0f) ? 1.0f : 0.0f;
        P.carry = P.gate;
    }
}

// The lane model's partials (gap = g0 + d_h - d, dv = v - v_h).
template <int MODE>
__device__ __forceinline__ void partials(const Veh &q, float d, float v, float dh, float vh,
                                         float dt, float inv_dt, float a_min, float gap_floor,
                                         Part &P) {
    partials_gd<MODE>(q, v, q.g0 + (dh - d), v - vh, dt, inv_dt, a_min, gap_floor, P);
}

__device__ __forceinline__ double block_sum(double x, double *red) {
    // fixed-order reduction: wave shuffles, then waves in index order
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = x;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) s += red[i];
    }
    __syncthreads();
    return s;
}

}  // namespace
}  // namespace idmx
