/*
 * FP64 CPU oracle of the differentiable Intelligent Driver Model simulator of
 * "Gradient-based Trajectory Optimization with Parallelized Differentiable
 * Traffic Simulation" (arXiv 2412.16750).
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library; the product (HIP) path
 * never links, loads or calls it, and the two share no code.
 *
 * Everything here is plain, sequential double-precision code that follows the
 * paper's definitions in the paper's order:
 *   - gap and speed difference to the leader h(i)        (Sec. III-A)
 *   - desired gap s_opt                                    (Sec. III-A, Eq. 1)
 *   - IDM acceleration                                     (Sec. III-A, Eq. 2)
 *   - explicit Euler update of position and speed          (Sec. III-A, Eq. 3)
 *   - synchronous per-frame update of all vehicles         (Sec. III-B, Fig. 3)
 *   - softplus lower bounds on s_opt and on a              (Sec. III-C)
 *   - trajectory loss over observed steps                  (Sec. IV-A, Eq. 4;
 *     squared error here, see below)
 * The reverse-mode gradient is derived by hand from those equations (the
 * paper obtains it by automatic differentiation, Sec. III-B / V): the adjoint
 * is the plain transpose of the per-step Jacobian, applied step by step from
 * the last step to the first, and scattered from each follower to its leader.
 *
 * Readings where the paper is silent:
 *   - Two velocity bounds.  MODE_SOFTPLUS is the paper's Sec. III-C
 *     (s* = softplus(s_opt); a* = a_lb + softplus(a - a_lb) with
 *     a_lb = max(-v/dt, a_min)).  MODE_CLAMP is the textbook IDM with the
 *     speed clamped at zero after the update: v' = max(v + dt*a, 0).
 *   - The lane head has no leader: it drives on a free road, i.e. the
 *     interaction term (s/gap)^2 is zero.
 *   - The gap used in (s/gap)^2 is floored at gap_floor (gradient zero where
 *     the floor is active); the forward returns how often it was active.
 *   - At a tie -v/dt == a_min the a_min branch (derivative 0) is taken.
 *   - (v/v0)^delta is evaluated as |v/v0|^delta.
 *   - The loss is the mean squared error over the observed (step, vehicle)
 *     pairs instead of the paper's summed absolute error (the MAE variant is a
 *     separate function).
 *
 * Layout: vehicles are grouped in lanes (CSR offsets lane_off[0..L]); inside a
 * lane they are ordered head -> tail, so the leader of vehicle i is i-1 unless
 * i is the first vehicle of its lane.  Arrays over time are step-major:
 * X[k*n + i] is vehicle i at step k, k = 0..n_steps.
 * Parameter arrays are ordered (v0, T, a, b, s0) = (v_targ, T_pref, a_max,
 * a_pref, s_min) in the paper's notation.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MODE_SOFTPLUS 0
#define MODE_CLAMP 1

typedef struct {
    int mode;
    double dt, delta, a_min, gap_floor;
} cfg_t;

/* Sec. III-C: softplus(x) = log(1 + exp(x)), written in its overflow-free form. */
static double softplus(double x) { return fmax(x, 0.0) + log1p(exp(-fabs(x))); }

/* d softplus(x) / dx */
static double logistic(double x)
{
    if (x >= 0.0) return 1.0 / (1.0 + exp(-x));
    double e = exp(x);
    return e / (1.0 + e);
}

/* One vehicle at one step: the acceleration that enters the speed update, and
 * (if want) its partial derivatives with respect to own position p, own speed
 * v, leader position ph, leader speed vh and the five parameters. */
typedef struct {
    double acc;
    double d_p, d_v, d_ph, d_vh;
    double d_prm[5]; /* v0, T, a, b, s0 */
    int floor_active;
    double ahat;     /* Eq. 2 before the Sec. III-C bound / the speed clamp */
    double gap;      /* raw bumper-to-bumper gap; +inf without a leader */
} local_t;

static local_t idm_local(const cfg_t *c, int has_leader, double p, double v, double ph,
                         double vh, double len_h, double v0, double T, double a, double b,
                         double s0, int want)
{
    local_t r;
    memset(&r, 0, sizeof r);

    /* free-road term (v / v0)^delta, Eq. 2 */
    double x = v / v0;
    double xd = pow(fabs(x), c->delta);
    double dxd_dx = (c->delta == 0.0) ? 0.0 : c->delta * pow(fabs(x), c->delta - 1.0) * (x < 0 ? -1.0 : 1.0);

    r.gap = INFINITY;
    double inter = 0.0;              /* (s* / gap)^2 */
    double dI_ds = 0.0, dI_dgap = 0.0; /* partials of inter w.r.t. s_opt and raw gap */
    double ds_dv = 0.0, ds_dvh = 0.0, ds_dT = 0.0, ds_da = 0.0, ds_db = 0.0, ds_ds0 = 0.0;
    if (has_leader) {
        /* Sec. III-A: gap and speed difference */
        double gap = ph - p - len_h;
        double dv = v - vh;
        r.gap = gap;
        double sg = gap > c->gap_floor ? gap : c->gap_floor;
        r.floor_active = !(gap > c->gap_floor);
        /* Eq. 1 */
        double root = sqrt(a * b);
        double s_opt = s0 + v * T + v * dv / (2.0 * root);
        double s_star = s_opt, ds_star = 1.0;
        if (c->mode == MODE_SOFTPLUS) { /* Sec. III-C: lower bound 0 on s_opt */
            s_star = softplus(s_opt);
            ds_star = logistic(s_opt);
        }
        double q = s_star / sg;
        inter = q * q;
        /* derivatives of inter */
        dI_ds = 2.0 * q / sg * ds_star;                     /* d inter / d s_opt */
        dI_dgap = r.floor_active ? 0.0 : -2.0 * q * q / sg; /* d inter / d gap   */
        /* derivatives of s_opt */
        ds_dv = T + (dv + v) / (2.0 * root);
        ds_dvh = -v / (2.0 * root);
        ds_dT = v;
        ds_ds0 = 1.0;
        /* d/da of 1/(2 sqrt(ab)) = -1/(4 a sqrt(ab)); same for b */
        ds_da = -v * dv / (4.0 * a * root);
        ds_db = -v * dv / (4.0 * b * root);
    }

    /* Eq. 2 */
    double ahat = a * (1.0 - xd - inter);
    r.ahat = ahat;
    /* partials of ahat */
    double h_v = a * (-dxd_dx / v0 - dI_ds * ds_dv);
    double h_vh = -a * dI_ds * ds_dvh;
    double h_gap = -a * dI_dgap; /* gap = ph - p - len_h */
    double h_v0 = a * dxd_dx * x / v0;
    double h_T = -a * dI_ds * ds_dT;
    double h_a = (1.0 - xd - inter) - a * dI_ds * ds_da;
    double h_b = -a * dI_ds * ds_db;
    double h_s0 = -a * dI_ds * ds_ds0;

    double w = 1.0, dlb_dv = 0.0, acc = ahat;
    if (c->mode == MODE_SOFTPLUS) {
        /* Sec. III-C: a* = a_lb + softplus(a - a_lb), a_lb = max(-v/dt, a_min) */
        double a_lb = -v / c->dt;
        if (a_lb > c->a_min) {
            dlb_dv = -1.0 / c->dt;
        } else {
            a_lb = c->a_min;
        }
        acc = a_lb + softplus(ahat - a_lb);
        w = logistic(ahat - a_lb);
    }
    r.acc = acc;
    if (want) {
        r.d_v = w * h_v + (1.0 - w) * dlb_dv;
        r.d_vh = w * h_vh;
        r.d_ph = w * h_gap;
        r.d_p = -w * h_gap;
        r.d_prm[0] = w * h_v0;
        r.d_prm[1] = w * h_T;
        r.d_prm[2] = w * h_a;
        r.d_prm[3] = w * h_b;
        r.d_prm[4] = w * h_s0;
    }
    return r;
}

/* Speed after one Euler step (Eq. 3) with the mode's bound, and the gate
 * d v' / d (v + dt*acc) (1 for SOFTPLUS, the clamp indicator for CLAMP). */
static double speed_update(const cfg_t *c, double v, double acc, double *gate)
{
    double vn = v + c->dt * acc;
    if (c->mode == MODE_CLAMP) {
        if (vn > 0.0) {
            *gate = 1.0;
        } else {
            *gate = 0.0;
            vn = 0.0;
        }
    } else {
        *gate = 1.0;
    }
    return vn;
}

static int check_common(const cfg_t *c, int n, int n_lanes, const int *lane_off, int n_steps)
{
    if (n < 0 || n_lanes < 0 || n_steps < 0 || !lane_off) return -1;
    if (!(c->dt > 0.0) || !(c->gap_floor >= 0.0)) return -1;
    if (c->mode != MODE_SOFTPLUS && c->mode != MODE_CLAMP) return -1;
    if (lane_off[0] != 0 || lane_off[n_lanes] != n) return -1;
    for (int l = 0; l < n_lanes; ++l)
        if (lane_off[l + 1] < lane_off[l]) return -1;
    return 0;
}

/*
 * Forward simulation.  P and V receive positions and speeds for steps
 * 0..n_steps ([(n_steps+1)*n]); A (nullable) receives the acceleration that
 * entered each update ([n_steps*n]; for MODE_CLAMP the effective (v'-v)/dt).
 * Lanes are independent (the leader relation never crosses a lane), so each
 * lane is simulated on its own, all steps at once.  Inside a step every
 * vehicle first reads the step-k state, then all are updated (Sec. III-B).
 * Returns the number of (vehicle, step) evaluations with the gap floor
 * active, or -1 on invalid arguments.
 */
long oracle_forward(int mode, double dt, double delta, double a_min, double gap_floor,
                    int n, int n_lanes, const int *lane_off, int n_steps,
                    const double *v0, const double *T, const double *a, const double *b,
                    const double *s0, const double *len, const double *p_init,
                    const double *v_init, double *P, double *V, double *A)
{
    cfg_t c = {mode, dt, delta, a_min, gap_floor};
    if (check_common(&c, n, n_lanes, lane_off, n_steps)) return -1;
    long floor_hits = 0;
    double *acc = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!acc) return -1;
    for (int i = 0; i < n; ++i) {
        P[i] = p_init[i];
        V[i] = v_init[i];
    }
    for (int l = 0; l < n_lanes; ++l) {
        int lo = lane_off[l], hi = lane_off[l + 1];
        for (int k = 0; k < n_steps; ++k) {
            const double *Pk = P + (size_t)k * n, *Vk = V + (size_t)k * n;
            double *Pn = P + (size_t)(k + 1) * n, *Vn = V + (size_t)(k + 1) * n;
            /* gather: every vehicle reads step-k values of itself and its leader */
            for (int i = lo; i < hi; ++i) {
                int has = i > lo;
                int h = has ? i - 1 : i;
                local_t r = idm_local(&c, has, Pk[i], Vk[i], Pk[h], Vk[h], len[h], v0[i], T[i],
                                      a[i], b[i], s0[i], 0);
                acc[i] = r.acc;
                floor_hits += r.floor_active;
            }
            /* update (Eq. 3): position with the old speed, then speed */
            for (int i = lo; i < hi; ++i) {
                double gate;
                Pn[i] = Pk[i] + dt * Vk[i];
                Vn[i] = speed_update(&c, Vk[i], acc[i], &gate);
                if (A) A[(size_t)k * n + i] = (mode == MODE_CLAMP) ? (Vn[i] - Vk[i]) / dt : acc[i];
            }
        }
    }
    free(acc);
    return floor_hits;
}

/*
 * Test helper: for every step k < n_steps and vehicle i of a forward
 * trajectory P, V, the quantities that decide the branches of the bounds:
 * AH = the IDM acceleration of Eq. 2 before the Sec. III-C bound or the speed
 * clamp, GAP = the raw bumper-to-bumper gap to the leader (+inf for a lane
 * head).  Both [n_steps * n].  A test uses them to tell how far each
 * evaluation is from a kink (a_lb switching branch, the clamp, the gap floor).
 */
int oracle_branch_terms(int mode, double dt, double delta, double a_min, double gap_floor,
                        int n, int n_lanes, const int *lane_off, int n_steps,
                        const double *v0, const double *T, const double *a, const double *b,
                        const double *s0, const double *len, const double *P, const double *V,
                        double *AH, double *GAP)
{
    cfg_t c = {mode, dt, delta, a_min, gap_floor};
    if (check_common(&c, n, n_lanes, lane_off, n_steps)) return -1;
    for (int l = 0; l < n_lanes; ++l) {
        int lo = lane_off[l], hi = lane_off[l + 1];
        for (int k = 0; k < n_steps; ++k) {
            const double *Pk = P + (size_t)k * n, *Vk = V + (size_t)k * n;
            for (int i = lo; i < hi; ++i) {
                int has = i > lo;
                int h = has ? i - 1 : i;
                local_t r = idm_local(&c, has, Pk[i], Vk[i], Pk[h], Vk[h], len[h], v0[i], T[i],
                                      a[i], b[i], s0[i], 0);
                AH[(size_t)k * n + i] = r.ahat;
                GAP[(size_t)k * n + i] = r.gap;
            }
        }
    }
    return 0;
}

/*
 * Reverse-mode gradient.  Inputs: the forward trajectory P, V, and the
 * upstream gradients gP = dL/dp_k ([(n_steps+1)*n]) and gV = dL/dv_k
 * (nullable, same shape).  Outputs (overwritten): g_prm [5*n] (v0, T, a, b,
 * s0 blocks of n), g_p0 [n] = dL/dp(0), g_v0 [n] = dL/dv(0), and, if g_abs
 * is non-null, g_abs [5*n] = the sum over steps of |mu_i d acc_i/d theta_i|,
 * the magnitude of the terms each parameter gradient adds up (a gradient far
 * smaller than it is a cancelling sum, which no FP32 trajectory determines to
 * a fixed relative accuracy).
 *
 * Per step k (last to first), with lam_p, lam_v the adjoints of the step-(k+1)
 * state and acc = f(p_i, v_i, p_h, v_h, theta_i):
 *   p_i(k+1) = p_i + dt v_i,  v_i(k+1) = bound(v_i + dt acc_i)
 *   lam_p(k)[i] += lam_p[i] + mu_i d acc_i/d p_i ;  lam_p(k)[h] += mu_i d acc_i/d p_h
 *   lam_v(k)[i] += dt lam_p[i] + g_i lam_v[i] + mu_i d acc_i/d v_i ;
 *   lam_v(k)[h] += mu_i d acc_i/d v_h ;  g_theta_i += mu_i d acc_i/d theta_i
 * with g_i the bound's gate and mu_i = g_i dt lam_v[i].
 */
int oracle_adjoint(int mode, double dt, double delta, double a_min, double gap_floor,
                   int n, int n_lanes, const int *lane_off, int n_steps,
                   const double *v0, const double *T, const double *a, const double *b,
                   const double *s0, const double *len, const double *P, const double *V,
                   const double *gP, const double *gV, double *g_prm, double *g_p0,
                   double *g_v0, double *g_abs)
{
    cfg_t c = {mode, dt, delta, a_min, gap_floor};
    if (check_common(&c, n, n_lanes, lane_off, n_steps)) return -1;
    size_t nn = (size_t)(n > 0 ? n : 1);
    double *lp = (double *)calloc(nn, sizeof(double)), *lv = (double *)calloc(nn, sizeof(double));
    double *np_ = (double *)calloc(nn, sizeof(double)), *nv = (double *)calloc(nn, sizeof(double));
    if (!lp || !lv || !np_ || !nv) {
        free(lp); free(lv); free(np_); free(nv);
        return -1;
    }
    for (int j = 0; j < 5 * n; ++j) g_prm[j] = 0.0;
    if (g_abs)
        for (int j = 0; j < 5 * n; ++j) g_abs[j] = 0.0;
    for (int i = 0; i < n; ++i) {
        lp[i] = gP[(size_t)n_steps * n + i];
        lv[i] = gV ? gV[(size_t)n_steps * n + i] : 0.0;
    }
    for (int k = n_steps - 1; k >= 0; --k) {
        const double *Pk = P + (size_t)k * n, *Vk = V + (size_t)k * n;
        for (int i = 0; i < n; ++i) {
            np_[i] = gP[(size_t)k * n + i] + lp[i];
            nv[i] = (gV ? gV[(size_t)k * n + i] : 0.0) + dt * lp[i];
        }
        for (int l = 0; l < n_lanes; ++l) {
            int lo = lane_off[l], hi = lane_off[l + 1];
            for (int i = lo; i < hi; ++i) {
                int has = i > lo;
                int h = has ? i - 1 : i;
                local_t r = idm_local(&c, has, Pk[i], Vk[i], Pk[h], Vk[h], len[h], v0[i], T[i],
                                      a[i], b[i], s0[i], 1);
                double gate;
                (void)speed_update(&c, Vk[i], r.acc, &gate);
                double mu = gate * dt * lv[i];
                nv[i] += gate * lv[i] + mu * r.d_v;
                np_[i] += mu * r.d_p;
                if (has) { /* scatter to the leader */
                    np_[h] += mu * r.d_ph;
                    nv[h] += mu * r.d_vh;
                }
                for (int j = 0; j < 5; ++j) g_prm[(size_t)j * n + i] += mu * r.d_prm[j];
                if (g_abs)
                    for (int j = 0; j < 5; ++j) g_abs[(size_t)j * n + i] += fabs(mu * r.d_prm[j]);
            }
        }
        memcpy(lp, np_, sizeof(double) * (size_t)n);
        memcpy(lv, nv, sizeof(double) * (size_t)n);
    }
    for (int i = 0; i < n; ++i) {
        g_p0[i] = lp[i];
        g_v0[i] = lv[i];
    }
    free(lp); free(lv); free(np_); free(nv);
    return 0;
}

/*
 * Tangent-linear (forward-mode) derivative: given directions dprm [5*n],
 * dp0 [n], dv0 [n], writes dP, dV [(n_steps+1)*n] = the directional derivative
 * of the trajectory.  Uses the same local partials as the adjoint but applies
 * them forward in time; a dot-product test between the two checks that the
 * adjoint is the exact transpose.
 */
int oracle_tangent(int mode, double dt, double delta, double a_min, double gap_floor,
                   int n, int n_lanes, const int *lane_off, int n_steps,
                   const double *v0, const double *T, const double *a, const double *b,
                   const double *s0, const double *len, const double *P, const double *V,
                   const double *dprm, const double *dp0, const double *dv0, double *dP,
                   double *dV)
{
    cfg_t c = {mode, dt, delta, a_min, gap_floor};
    if (check_common(&c, n, n_lanes, lane_off, n_steps)) return -1;
    for (int i = 0; i < n; ++i) {
        dP[i] = dp0[i];
        dV[i] = dv0[i];
    }
    for (int k = 0; k < n_steps; ++k) {
        const double *Pk = P + (size_t)k * n, *Vk = V + (size_t)k * n;
        const double *dPk = dP + (size_t)k * n, *dVk = dV + (size_t)k * n;
        double *dPn = dP + (size_t)(k + 1) * n, *dVn = dV + (size_t)(k + 1) * n;
        for (int l = 0; l < n_lanes; ++l) {
            int lo = lane_off[l], hi = lane_off[l + 1];
            for (int i = lo; i < hi; ++i) {
                int has = i > lo;
                int h = has ? i - 1 : i;
                local_t r = idm_local(&c, has, Pk[i], Vk[i], Pk[h], Vk[h], len[h], v0[i], T[i],
                                      a[i], b[i], s0[i], 1);
                double gate;
                (void)speed_update(&c, Vk[i], r.acc, &gate);
                double dacc = r.d_p * dPk[i] + r.d_v * dVk[i];
                if (has) dacc += r.d_ph * dPk[h] + r.d_vh * dVk[h];
                for (int j = 0; j < 5; ++j) dacc += r.d_prm[j] * dprm[(size_t)j * n + i];
                dPn[i] = dPk[i] + dt * dVk[i];
                dVn[i] = gate * (dVk[i] + dt * dacc);
            }
        }
    }
    return 0;
}

/*
 * Mean squared trajectory error over observed steps (the squared-error
 * counterpart of Sec. IV-A, Eq. 4): for observed step list steps[0..n_obs-1]
 * and targets target[j*n + i] (absolute positions),
 *   L = 1/(n_obs*n) * sum_j sum_i (P[steps[j]*n + i] - target[j*n + i])^2.
 * If gP is non-null, dL/dP is ADDED into it ([(n_steps+1)*n]).
 */
double oracle_mse(int n, int n_steps, const double *P, int n_obs, const int *steps,
                  const double *target, double *gP)
{
    if (n <= 0 || n_obs <= 0) return 0.0;
    double sum = 0.0, inv = 1.0 / ((double)n_obs * (double)n);
    for (int j = 0; j < n_obs; ++j) {
        int k = steps[j];
        if (k < 0 || k > n_steps) return NAN;
        for (int i = 0; i < n; ++i) {
            double r = P[(size_t)k * n + i] - target[(size_t)j * n + i];
            sum += r * r;
            if (gP) gP[(size_t)k * n + i] += 2.0 * r * inv;
        }
    }
    return sum * inv;
}

/*
 * The paper's reconstruction loss (Sec. IV-A, Eq. 4): sum over observed
 * pairs of |P_obs - P[k]|.  Subgradient sign(r) (0 at r == 0) is ADDED into gP.
 */
double oracle_mae_sum(int n, int n_steps, const double *P, int n_obs, const int *steps,
                      const double *target, double *gP)
{
    double sum = 0.0;
    for (int j = 0; j < n_obs; ++j) {
        int k = steps[j];
        if (k < 0 || k > n_steps) return NAN;
        for (int i = 0; i < n; ++i) {
            double r = P[(size_t)k * n + i] - target[(size_t)j * n + i];
            sum += fabs(r);
            if (gP) gP[(size_t)k * n + i] += (r > 0.0) - (r < 0.0);
        }
    }
    return sum;
}

/* ------------------------------------------------------------------------
 * Ego-only reconstruction (Sec. IV-A, trajectory filtering / reconstruction).
 * Every trajectory i is one vehicle whose leader is not simulated: at each
 * step k its bumper-to-bumper gap G[k*n+i] and its speed difference
 * D[k*n+i] = v - v_h to the (unobserved) leader are free variables of the
 * fit, and p(0) = 0.  The loss is the paper's summed absolute error between
 * the observed positions and the simulated position at the nearest step.
 *
 * The leader relation enters Eqs. 1-2 only through (gap, v - v_h), so one ego
 * step is the lane step of idm_local with a virtual leader of length 0 at
 * p_h = gap (own position 0) and speed v_h = v - D.  Its partials map as
 *   d acc / d G = d acc / d p_h,   d acc / d D = -d acc / d v_h,
 *   d acc / d v (D fixed) = d acc / d v + d acc / d v_h,
 * and the own position does not enter (the gap is given, not p_h - p).
 * ------------------------------------------------------------------------ */
static local_t ego_local(const cfg_t *c, double v, double gap, double dv, double v0, double T,
                         double a, double b, double s0, int want)
{
    return idm_local(c, 1, 0.0, v, gap, v - dv, 0.0, v0, T, a, b, s0, want);
}

static int ego_check(const cfg_t *c, int n, int n_steps)
{
    if (n < 0 || n_steps < 0) return -1;
    if (!(c->dt > 0.0) || !(c->gap_floor >= 0.0)) return -1;
    if (c->mode != MODE_SOFTPLUS && c->mode != MODE_CLAMP) return -1;
    return 0;
}

/*
 * Ego forward: P, V [(n_steps+1)*n] (P(0) = 0, V(0) = v_init), A (nullable)
 * [n_steps*n] the acceleration of each update (CLAMP: (v'-v)/dt).  Returns the
 * number of steps with the gap floor active, or -1 on invalid arguments.
 */
long oracle_ego_forward(int mode, double dt, double delta, double a_min, double gap_floor,
                        int n, int n_steps, const double *v0, const double *T, const double *a,
                        const double *b, const double *s0, const double *G, const double *D,
                        const double *v_init, double *P, double *V, double *A)
{
    cfg_t c = {mode, dt, delta, a_min, gap_floor};
    if (ego_check(&c, n, n_steps)) return -1;
    long hits = 0;
    for (int i = 0; i < n; ++i) {
        P[i] = 0.0;
        V[i] = v_init[i];
        for (int k = 0; k < n_steps; ++k) {
            size_t at = (size_t)k * n + i, nx = (size_t)(k + 1) * n + i;
            local_t r = ego_local(&c, V[at], G[at], D[at], v0[i], T[i], a[i], b[i], s0[i], 0);
            double gate;
            hits += r.floor_active;
            P[nx] = P[at] + dt * V[at];                      /* Eq. 3, old speed */
            V[nx] = speed_update(&c, V[at], r.acc, &gate);
            if (A) A[at] = (mode == MODE_CLAMP) ? (V[nx] - V[at]) / dt : r.acc;
        }
    }
    return hits;
}

/*
 * Ego adjoint for the upstream gP = dL/dP [(n_steps+1)*n].  Outputs
 * (overwritten): g_prm [5*n] (v0, T, a, b, s0), gG, gD [n_steps*n] (the
 * per-step free variables), g_v0 [n] = dL/dv(0).
 */
int oracle_ego_adjoint(int mode, double dt, double delta, double a_min, double gap_floor,
                       int n, int n_steps, const double *v0, const double *T, const double *a,
                       const double *b, const double *s0, const double *G, const double *D,
                       const double *P, const double *V, const double *gP, double *g_prm,
                       double *gG, double *gD, double *g_v0)
{
    cfg_t c = {mode, dt, delta, a_min, gap_floor};
    if (ego_check(&c, n, n_steps)) return -1;
    (void)P;
    for (int i = 0; i < n; ++i) {
        double lp = gP[(size_t)n_steps * n + i], lv = 0.0;
        double g[5] = {0, 0, 0, 0, 0};
        for (int k = n_steps - 1; k >= 0; --k) {
            size_t at = (size_t)k * n + i;
            local_t r = ego_local(&c, V[at], G[at], D[at], v0[i], T[i], a[i], b[i], s0[i], 1);
            double gate;
            (void)speed_update(&c, V[at], r.acc, &gate);
            double mu = gate * dt * lv;
            gG[at] = mu * r.d_ph;
            gD[at] = -mu * r.d_vh;
            for (int j = 0; j < 5; ++j) g[j] += mu * r.d_prm[j];
            double nlv = dt * lp + gate * lv + mu * (r.d_v + r.d_vh);
            lp = gP[at] + lp;
            lv = nlv;
        }
        for (int j = 0; j < 5; ++j) g_prm[(size_t)j * n + i] = g[j];
        g_v0[i] = lv;
    }
    return 0;
}

/*
 * Ego tangent-linear model: directions dprm [5*n], dG, dD [n_steps*n],
 * dv0 [n] -> dP, dV [(n_steps+1)*n] (dP(0) = 0).  The adjoint is its exact
 * transpose (dot-product test).
 */
int oracle_ego_tangent(int mode, double dt, double delta, double a_min, double gap_floor,
                       int n, int n_steps, const double *v0, const double *T, const double *a,
                       const double *b, const double *s0, const double *G, const double *D,
                       const double *V, const double *dprm, const double *dG,
                       const double *dD, const double *dv0, double *dP, double *dV)
{
    cfg_t c = {mode, dt, delta, a_min, gap_floor};
    if (ego_check(&c, n, n_steps)) return -1;
    for (int i = 0; i < n; ++i) {
        dP[i] = 0.0;
        dV[i] = dv0[i];
        for (int k = 0; k < n_steps; ++k) {
            size_t at = (size_t)k * n + i, nx = (size_t)(k + 1) * n + i;
            local_t r = ego_local(&c, V[at], G[at], D[at], v0[i], T[i], a[i], b[i], s0[i], 1);
            double gate;
            (void)speed_update(&c, V[at], r.acc, &gate);
            double dacc = (r.d_v + r.d_vh) * dV[at] + r.d_ph * dG[at] - r.d_vh * dD[at];
            for (int j = 0; j < 5; ++j) dacc += r.d_prm[j] * dprm[(size_t)j * n + i];
            dP[nx] = dP[at] + dt * dV[at];
            dV[nx] = gate * (dV[at] + dt * dacc);
        }
    }
    return 0;
}

/*
 * The reconstruction loss (Sec. IV-A): for trajectory i with observations
 * j = obs_off[i] .. obs_off[i+1]-1 at steps obs_step[j] (the nearest
 * simulation step of each timestamp) and positions obs_pos[j],
 *   L = sum_i sum_j |obs_pos[j] - P[obs_step[j]*n + i]|.
 * Subgradient sign(P - obs) (0 at equality) is ADDED into gP.  Returns NAN
 * for a step outside 0..n_steps.
 */
double oracle_ego_mae(int n, int n_steps, const double *P, const int *obs_off,
                      const int *obs_step, const double *obs_pos, double *gP)
{
    double sum = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int j = obs_off[i]; j < obs_off[i + 1]; ++j) {
            int k = obs_step[j];
            if (k < 0 || k > n_steps) return NAN;
            double r = P[(size_t)k * n + i] - obs_pos[j];
            sum += fabs(r);
            if (gP) gP[(size_t)k * n + i] += (r > 0.0) - (r < 0.0);
        }
    }
    return sum;
}
