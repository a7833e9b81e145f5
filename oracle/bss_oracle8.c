/*
 * bss_oracle8.c -- the paper's 8-state vehicle in the FP64 CPU oracle (vehicle = 1).
 *
 * TEST INFRASTRUCTURE ONLY, like bss_oracle.c: loaded by the tests, the smoke check and the
 * benchmark's CPU baseline; it shares no code with the GPU library.
 *
 * The Simulation Study models the AutoRally with the planar single-track vehicle of its Fig. 2:
 * state x = [vX, vY, r, wF, wR, epsi, eY, s] (body-frame velocities, yaw rate, front and rear
 * wheel speeds, heading error and lateral deviation from the centerline, path coordinate in the
 * road-aligned frame), input u = [steer, throttle], Pacejka tires with the friction ellipse for
 * combined slip.  It does not print the equations or the tire, wheel and track data; this file
 * writes out the standard form of that model (readings stated at each function) and the problem
 * builders state the generic coefficients used.  The rest of Alg. 1 / Alg. 2 is unchanged: the
 * belief is the Monte-Carlo mean of the 8 states and the variance of eY (eY is a state, so the
 * spread of eq. 11 along eta = grad c is the variance of eY itself), the barrier is eq. 33, the
 * running cost eq. 27 with Q over the 8 states, and the update eqs. 6-7 (orc_update).
 */
#include "bss_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

static double clamp8(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* Pacejka's magic formula for pure slip: D sin(C atan(B z - E (B z - atan(B z)))). */
double orc8_magic(const orc_params* p, double z)
{
    double bz = p->pac_B * z;
    return p->pac_D * sin(p->pac_C * atan(bz - p->pac_E * (bz - atan(bz))));
}

/* Forces of one tire in its own frame, F = (Fx, Fy), from the normal load Fz, the longitudinal
 * slip and the slip angle.  Pure slip: Fx0 = mu Fz MF(slip), Fy0 = mu Fz MF(alpha).  Combined slip
 * by the friction ellipse (reading): the longitudinal force is kept and the lateral force takes
 * what the ellipse of semi-axes Fmax = mu D Fz leaves, Fy = Fy0 sqrt(1 - (Fx0 / Fmax)^2), so the
 * combined force never leaves the ellipse and either pure-slip case is reproduced exactly. */
void orc8_tire(const orc_params* p, double Fz, double slip, double alpha, double F[2])
{
    double fmax = p->mu * p->pac_D * Fz;
    double fx0 = p->mu * Fz * orc8_magic(p, slip);
    double fy0 = p->mu * Fz * orc8_magic(p, alpha);
    double ratio = fmax > 0.0 ? fx0 / fmax : 0.0;
    double rem = 1.0 - ratio * ratio;
    F[0] = fx0;
    F[1] = fy0 * sqrt(rem > 0.0 ? rem : 0.0);
}

/* Centerline curvature of the synthetic closed track (reading: the AutoRally track is not
 * available): kappa(s) = (2 pi / L)(1 + a sin(4 pi s / L)); it turns by 2 pi over one lap of
 * length L, with two tighter and two gentler bends. */
double orc8_kappa(const orc_params* p, double s)
{
    double L = p->track_len;
    return (2.0 * M_PI / L) * (1.0 + p->kappa_amp * sin(4.0 * M_PI * s / L));
}

/* Vector field of the 8-state single-track vehicle.
 * Wheel-frame velocities: front (vX cos d + (vY + lf r) sin d, -vX sin d + (vY + lf r) cos d),
 * rear (vX, vY - lr r); longitudinal slip (Rw w - v_x) / max(v_x, v_min) and slip angle
 * -atan(v_y / max(v_x, v_min)) per axle; static normal loads m g lr / L and m g lf / L.
 * Body:   m (vX' - r vY) = Fxf cos d - Fyf sin d + Fxr
 *         m (vY' + r vX) = Fxf sin d + Fyf cos d + Fyr
 *         Iz r'          = lf (Fxf sin d + Fyf cos d) - lr Fyr
 * Wheels: Iw wF' = -Rw Fxf (front not driven),  Iw wR' = throttle T_max - Rw Fxr
 * Road-aligned frame (curvature kappa(s), eY positive to the left):
 *         s' = (vX cos epsi - vY sin epsi) / (1 - kappa eY)
 *         eY' = vX sin epsi + vY cos epsi,    epsi' = r - kappa s' */
void orc8_deriv(const orc_params* p, const double x[8], const double u[2], double dx[8])
{
    double vX = x[0], vY = x[1], r = x[2], wF = x[3], wR = x[4], epsi = x[5], eY = x[6];
    double s = x[7];
    double d = u[0], thr = u[1];
    double L = p->lf + p->lr;
    double Fzf = p->m * p->g * p->lr / L, Fzr = p->m * p->g * p->lf / L;
    double cd = cos(d), sd = sin(d);
    double vyf_b = vY + p->lf * r;
    double vxf = vX * cd + vyf_b * sd, vyf = -vX * sd + vyf_b * cd;
    double vxr = vX, vyr = vY - p->lr * r;
    double nf = vxf > p->v_min ? vxf : p->v_min, nr = vxr > p->v_min ? vxr : p->v_min;
    double Ff[2], Fr[2];
    orc8_tire(p, Fzf, (p->Rw * wF - vxf) / nf, -atan(vyf / nf), Ff);
    orc8_tire(p, Fzr, (p->Rw * wR - vxr) / nr, -atan(vyr / nr), Fr);
    double fx_body = Ff[0] * cd - Ff[1] * sd + Fr[0];
    double fy_front = Ff[0] * sd + Ff[1] * cd;
    dx[0] = r * vY + fx_body / p->m;
    dx[1] = -r * vX + (fy_front + Fr[1]) / p->m;
    dx[2] = (p->lf * fy_front - p->lr * Fr[1]) / p->Iz;
    dx[3] = -p->Rw * Ff[0] / p->Iw;
    dx[4] = (thr * p->T_max - p->Rw * Fr[0]) / p->Iw;
    double kap = orc8_kappa(p, s);
    double sdot = (vX * cos(epsi) - vY * sin(epsi)) / (1.0 - kap * eY);
    dx[5] = r - kap * sdot;
    dx[6] = vX * sin(epsi) + vY * cos(epsi);
    dx[7] = sdot;
}

/* One control period: n_sub explicit-midpoint substeps of dt / n_sub with the control held (the
 * wheel and tire dynamics are stiffer than one midpoint step of dt resolves). */
void orc8_step(const orc_params* p, const double x[8], const double u[2], double xn[8])
{
    int n = p->n_sub > 0 ? p->n_sub : 1;
    double h = p->dt / n;
    double cur[8], k1[8], xm[8], k2[8];
    memcpy(cur, x, sizeof(cur));
    for (int i = 0; i < n; ++i) {
        orc8_deriv(p, cur, u, k1);
        for (int j = 0; j < 8; ++j) xm[j] = cur[j] + 0.5 * h * k1[j];
        orc8_deriv(p, xm, u, k2);
        for (int j = 0; j < 8; ++j) cur[j] += h * k2[j];
    }
    memcpy(xn, cur, sizeof(cur));
}

/* Belief record of a particle set (the Monte-Carlo estimates of Alg. 2): the mean of the 8 states
 * and the unbiased variance of eY (two-pass; 0 for M = 1). */
void orc8_moments(const double* particles, int32_t M, double rec[9])
{
    for (int j = 0; j < 8; ++j) {
        double acc = 0.0;
        for (int m = 0; m < M; ++m) acc += particles[m * 8 + j];
        rec[j] = acc / M;
    }
    double var = 0.0;
    for (int m = 0; m < M; ++m) {
        double d = particles[m * 8 + 6] - rec[6];
        var += d * d;
    }
    rec[8] = M > 1 ? var / (M - 1) : 0.0;
}

/* eq. 33 with the clamp of the 6-state car: h = max(w_T - nu sigma_y, 0)^2 - eY_bar^2, sigma_y the
 * standard deviation of eY. */
double orc8_barrier(const orc_params* p, double nu, const double rec[9])
{
    double sig = sqrt(rec[8] > 0.0 ? rec[8] : 0.0);
    double margin = p->half_width - nu * sig;
    if (margin < 0.0) margin = 0.0;
    return margin * margin - rec[6] * rec[6];
}

/* eq. 27 on the mean: (x - x_g)^T Q (x - x_g) with x_g = (v_goal, 0, ..., 0) and Q = diag(q_vx,
 * q_vy, q_r, 0, 0, q_epsi, q_ey, 0), plus C_obs when the mean is outside the track. */
double orc8_stage_cost(const orc_params* p, const double rec[9])
{
    double dv = rec[0] - p->v_goal;
    double q = p->q_vx * dv * dv + p->q_vy * rec[1] * rec[1] + p->q_r * rec[2] * rec[2] +
               p->q_epsi * rec[5] * rec[5] + p->q_ey * rec[6] * rec[6];
    if (fabs(rec[6]) >= p->half_width) q += p->C_obs;
    return q;
}

/* The shield repair of the 6-state car (orc_repair) on this model: one-step residual
 * r(u) = -h(f(xbar_t, u); sigma_t) + (1 - gamma) h_t with the spread frozen at step t, damped
 * Gauss-Newton steps u <- clip(u - max(r, 0) g / (|g|^2 + gmin^2)), g by central differences. */
static double residual8(const orc_params* p, double nu, const double rec_t[9], double h_t,
                        const double u[2])
{
    double xn[9];
    orc8_step(p, rec_t, u, xn);
    xn[8] = rec_t[8];
    return -orc8_barrier(p, nu, xn) + (1.0 - p->gamma) * h_t;
}

void orc8_repair(const orc_params* p, double nu, const double rec_t[9], double u[2])
{
    if (p->shield_iters <= 0) return;
    double h_t = orc8_barrier(p, nu, rec_t);
    double fd = p->shield_fd;
    for (int it = 0; it < p->shield_iters; ++it) {
        double r0 = residual8(p, nu, rec_t, h_t, u);
        if (!(r0 > 0.0)) break;
        double g[2];
        for (int j = 0; j < 2; ++j) {
            double up[2] = {u[0], u[1]}, um[2] = {u[0], u[1]};
            up[j] += fd;
            um[j] -= fd;
            g[j] = (residual8(p, nu, rec_t, h_t, up) - residual8(p, nu, rec_t, h_t, um)) /
                   (2.0 * fd);
        }
        double den = g[0] * g[0] + g[1] * g[1] + p->shield_gmin * p->shield_gmin;
        u[0] = clamp8(u[0] - r0 * g[0] / den, -p->steer_max, p->steer_max);
        u[1] = clamp8(u[1] - r0 * g[1] / den, -p->accel_max, p->accel_max);
    }
}

/* Trajectory cost of one sample (Alg. 1), as orc_score: running cost at t = 0..T-1 with the
 * control cost, C_safe on every transition (0 at t = 0), terminal phi_scale times the running
 * cost. */
double orc8_score(const orc_params* p, double nu, const double* rec, const double* u,
                  const double* v)
{
    int T = p->T;
    double inv_var[2];
    for (int j = 0; j < 2; ++j)
        inv_var[j] = p->sigma_eps[j] > 0.0 ? 1.0 / (p->sigma_eps[j] * p->sigma_eps[j]) : 0.0;
    double S = 0.0;
    double h_prev = orc8_barrier(p, nu, &rec[0]);
    for (int t = 0; t < T; ++t) {
        const double* rt = &rec[(size_t)t * 9];
        double h_t = orc8_barrier(p, nu, rt);
        double c_safe = 0.0;
        if (t > 0) {
            double viol = -h_t + (1.0 - p->gamma) * h_prev;
            c_safe = p->C_cbf * (viol > 0.0 ? viol : 0.0);
        }
        double ctrl = p->gamma_u * (v[t * 2 + 0] * inv_var[0] * u[t * 2 + 0] +
                                    v[t * 2 + 1] * inv_var[1] * u[t * 2 + 1]);
        S += orc8_stage_cost(p, rt) + ctrl + c_safe;
        h_prev = h_t;
    }
    const double* rT = &rec[(size_t)T * 9];
    double h_T = orc8_barrier(p, nu, rT);
    double viol = -h_T + (1.0 - p->gamma) * h_prev;
    S += p->phi_scale * orc8_stage_cost(p, rT) + p->C_cbf * (viol > 0.0 ? viol : 0.0);
    return S;
}

/* Sample k: eps from tag 0 as for the 6-state car, u = clip(v + eps), the repair, then the M
 * particles (all starting at the estimate) pushed through orc8_step plus the disturbance on
 * (vX, vY, r) from the quad-dealt normals of tag 1 (orc_disturbance_normals). */
static double rollout8(const orc_params* p, double nu, uint32_t s, int32_t k, const double x0[8],
                       const double* v, double* u_out, double* rec_out)
{
    int M = p->M, T = p->T;
    double* part = (double*)malloc(sizeof(double) * 8 * (size_t)M);
    for (int m = 0; m < M; ++m) memcpy(&part[m * 8], x0, sizeof(double) * 8);
    orc8_moments(part, M, rec_out);
    uint32_t kw = p->crn ? 0u : (uint32_t)k;
    for (int t = 0; t < T; ++t) {
        uint32_t ctr[4] = {(uint32_t)t, 0u, (uint32_t)k, s & 0x0FFFFFFFu};
        double z[4];
        orc_normals(p->seed, ctr, z);
        double u[2];
        u[0] = clamp8(v[t * 2 + 0] + p->sigma_eps[0] * z[0], -p->steer_max, p->steer_max);
        u[1] = clamp8(v[t * 2 + 1] + p->sigma_eps[1] * z[1], -p->accel_max, p->accel_max);
        orc8_repair(p, nu, &rec_out[(size_t)t * 9], u);
        u_out[t * 2 + 0] = u[0];
        u_out[t * 2 + 1] = u[1];
        for (int m = 0; m < M; ++m) {
            double xn[8], w[3];
            orc8_step(p, &part[m * 8], u, xn);
            orc_disturbance_normals(p->seed, s, kw, (uint32_t)t, (uint32_t)m, w);
            for (int j = 0; j < 3; ++j) xn[j] += p->sigma_w[j] * w[j];
            memcpy(&part[m * 8], xn, sizeof(xn));
        }
        orc8_moments(part, M, &rec_out[(size_t)(t + 1) * 9]);
    }
    free(part);
    return orc8_score(p, nu, rec_out, u_out, v);
}

typedef struct {
    const orc_params* p;
    double nu;
    uint32_t s;
    const double* x0;
    const double* v;
    double *u, *rec, *S;
    int k_begin, k_end;
} job8;

static void* worker8(void* arg)
{
    job8* j = (job8*)arg;
    size_t T = (size_t)j->p->T;
    for (int k = j->k_begin; k < j->k_end; ++k)
        j->S[k] = rollout8(j->p, j->nu, j->s, k, j->x0, j->v, &j->u[(size_t)k * T * 2],
                           &j->rec[(size_t)k * (T + 1) * 9]);
    return NULL;
}

/* One solve of the 8-state problem (Alg. 1's body): all K rollouts, then the update of v in
 * place (orc_update).  The estimate x0 [8] is known exactly (no initial spread).  u_out
 * [K][T][2], rec_out [K][T+1][9] and S_out [K] may be NULL.  Returns 0, or 1 when no cost is
 * finite. */
int32_t orc8_solve(const orc_params* p, uint32_t s, const double x0[8], double* v, double* u_out,
                   double* rec_out, double* S_out, double stats[4], int32_t nthreads)
{
    int K = p->K, T = p->T;
    double nu = orc_backoff(p->delta, p->backoff);
    double* u = u_out ? u_out : (double*)malloc(sizeof(double) * (size_t)K * T * 2);
    double* rec = rec_out ? rec_out : (double*)malloc(sizeof(double) * (size_t)K * (T + 1) * 9);
    double* S = S_out ? S_out : (double*)malloc(sizeof(double) * (size_t)K);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > K) nthreads = K;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    job8* jobs = (job8*)malloc(sizeof(job8) * (size_t)nthreads);
    for (int i = 0; i < nthreads; ++i) {
        job8 j = {p, nu, s, x0, v, u, rec, S, (int)((long)K * i / nthreads),
                  (int)((long)K * (i + 1) / nthreads)};
        jobs[i] = j;
        if (nthreads == 1) worker8(&jobs[i]);
        else pthread_create(&th[i], NULL, worker8, &jobs[i]);
    }
    if (nthreads > 1)
        for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
    free(th);
    free(jobs);
    int32_t rc = orc_update(p, S, u, v, stats);
    if (!u_out) free(u);
    if (!rec_out) free(rec);
    if (!S_out) free(S);
    return rc;
}
