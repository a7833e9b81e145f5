/*
 * bss_oracle.c -- plain FP64 CPU oracle for BSS-MPPI (arXiv 2408.00494).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the benchmark's CPU
 * baseline.  It shares no code with the GPU library; it is written for readability, not speed.
 *
 * What each function follows in the paper:
 *   - orc_solve / orc_rollout / orc_score: Alg. 1 (sample M control sequences in parallel, roll
 *     each over the horizon, accumulate q + gamma v^T Sigma_eps^-1 u + C_safe per step, then the
 *     terminal phi + C_safe), with the belief propagated by Alg. 2 (Monte-Carlo particles).
 *   - orc_moments: the Monte-Carlo mean and unbiased covariance (the two displayed estimates
 *     that precede the augmented-system section, and the last two lines of Alg. 2).
 *   - orc_barrier: the application DCBF h = (w_T - nu sigma_y)^2 - e_y^2 (eq. 33) built from the
 *     deterministic chance constraint c(xbar) + nu sqrt(eta^T Sigma eta) <= 0 (eq. 11).
 *   - C_safe: eq. 25 with the linear class-kappa condition of eq. 24 (rate beta, here gamma).
 *   - orc_update: the MPPI update law (eq. 6) with the min-shifted weights (eq. 7).
 *   - orc_backoff: Remark 1 (Gaussian or Cantelli back-off coefficient).
 * Readings where the paper is silent (the car model, the track geometry, the repair, the
 * random-number contract) are stated next to the code that implements them.
 */
#include "bss_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ============================ Philox4x32-10 and Box-Muller ============================ */
/* Philox4x32 with 10 rounds as defined by Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3" (SC'11): each round multiplies counter words 0 and 2 by two fixed odd
 * constants, swaps the high/low halves into a permuted output and xors in the round key; the key
 * is advanced by two Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint64_t MULT0 = 0xD2511F53u, MULT1 = 0xCD9E8D57u;
    const uint32_t WEYL0 = 0x9E3779B9u, WEYL1 = 0xBB67AE85u;
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = MULT0 * (uint64_t)c[0];
        uint64_t p1 = MULT1 * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        uint32_t n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
        k0 += WEYL0;
        k1 += WEYL1;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* Uniform on (0,1) from the top 23 bits: ((r >> 9) + 1/2) * 2^-23.  Exactly representable in
 * single and double precision, never 0 or 1. */
double orc_uniform(uint32_t r)
{
    return ((double)(r >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* Four standard normals from one Philox block by the Box-Muller transform:
 * (r0, r1) -> rho0 (cos, sin)(2 pi u1); (r2, r3) -> rho2 (cos, sin)(2 pi u3). */
void orc_normals(uint64_t seed, const uint32_t ctr[4], double z[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    double u0 = orc_uniform(r[0]), u1 = orc_uniform(r[1]);
    double u2 = orc_uniform(r[2]), u3 = orc_uniform(r[3]);
    double rho0 = sqrt(-2.0 * log(u0));
    double rho2 = sqrt(-2.0 * log(u2));
    z[0] = rho0 * cos(2.0 * M_PI * u1);
    z[1] = rho0 * sin(2.0 * M_PI * u1);
    z[2] = rho2 * cos(2.0 * M_PI * u3);
    z[3] = rho2 * sin(2.0 * M_PI * u3);
}

/* Bulk helpers for tests: n counters ctr[n][4] -> out[n][4] words / normals. */
void orc_philox_many(const uint32_t* ctr, const uint32_t key[2], uint32_t* out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(&ctr[4 * i], key, &out[4 * i]);
}

void orc_normals_many(uint64_t seed, const uint32_t* ctr, double* z, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) orc_normals(seed, &ctr[4 * i], &z[4 * i]);
}

/* Counter layout (the random-number contract shared by both implementations):
 *   word0 = time step t (or the block index for the initial spread), word1 = particle m (for
 *   the disturbance: the block index 3q + b of particle quad q, see disturbance_normals),
 *   word2 = sample k, word3 = (stream tag << 28) | (solve index & 0x0FFFFFFF).
 * Tags: 0 control noise eps_{k,t}; 1 disturbance w_{k,m,t}; 2 initial spread of particles;
 * 4 and 5 the two blocks of standard normals of a Gaussian re-sampling draw (word0 = t). */
static void rng_counter(uint32_t w0, uint32_t m, uint32_t k, uint32_t tag, uint32_t s,
                        uint32_t ctr[4])
{
    ctr[0] = w0;
    ctr[1] = m;
    ctr[2] = k;
    ctr[3] = (tag << 28) | (s & 0x0FFFFFFFu);
}

/* ================================= back-off coefficient ================================= */
/* Remark 1: Gaussian nu = sqrt(2) erfinv(1 - 2 delta) = Phi^-1(1 - delta), found here by
 * bisection on the upper tail Q(x) = erfc(x / sqrt 2) / 2 = delta (the tail form keeps full relative
 * precision for small delta); Cantelli nu = sqrt((1 - delta) / delta). */
double orc_backoff(double delta, int32_t backoff)
{
    if (backoff == 1) return sqrt((1.0 - delta) / delta);
    double lo = -40.0, hi = 40.0;
    for (int it = 0; it < 2000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double tail = 0.5 * erfc(mid / sqrt(2.0));
        if (tail > delta) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* ======================================= dynamics ======================================= */
static double clampd(double x, double lo, double hi)
{
    return x < lo ? lo : (x > hi ? hi : x);
}

/* Single-track car with linear tires (the paper's plant is a single-track model; its tire and
 * mass data are not given, so this 6-state linear-tire variant is the stated substitute).
 * x = [X, Y, psi, vx, vy, r] (global position, heading, body-frame velocities, yaw rate),
 * u = [steer, accel].  Slip angles use max(vx, v_min); lateral forces saturate at the static
 * axle load times mu. */
void orc_car_deriv(const orc_params* p, const double x[6], const double u[2], double dx[6])
{
    double psi = x[2], vx = x[3], vy = x[4], r = x[5];
    double steer = u[0], accel = u[1];
    double vxs = vx > p->v_min ? vx : p->v_min;
    double alpha_f = steer - atan((vy + p->lf * r) / vxs);
    double alpha_r = -atan((vy - p->lr * r) / vxs);
    double wheelbase = p->lf + p->lr;
    double Ff_max = p->mu * p->m * p->g * p->lr / wheelbase;
    double Fr_max = p->mu * p->m * p->g * p->lf / wheelbase;
    double Ff = clampd(p->Cf * alpha_f, -Ff_max, Ff_max);
    double Fr = clampd(p->Cr * alpha_r, -Fr_max, Fr_max);
    dx[0] = vx * cos(psi) - vy * sin(psi);
    dx[1] = vx * sin(psi) + vy * cos(psi);
    dx[2] = r;
    dx[3] = accel + vy * r - Ff * sin(steer) / p->m;
    dx[4] = (Ff * cos(steer) + Fr) / p->m - vx * r;
    dx[5] = (p->lf * Ff * cos(steer) - p->lr * Fr) / p->Iz;
}

/* One discrete step of the noise-free model.  Car: explicit midpoint rule (RK2),
 * x+ = x + dt f(x + dt/2 f(x, u), u), zero-order hold on u.  Linear test model: x+ = A x + B u. */
void orc_model_step(const orc_params* p, const double x[6], const double u[2], double xn[6])
{
    if (p->model == 1) {
        for (int i = 0; i < 6; ++i) {
            double acc = 0.0;
            for (int j = 0; j < 6; ++j) acc += p->lin_A[i * 6 + j] * x[j];
            for (int j = 0; j < 2; ++j) acc += p->lin_B[i * 2 + j] * u[j];
            xn[i] = acc;
        }
        return;
    }
    double k1[6], xm[6], k2[6];
    orc_car_deriv(p, x, u, k1);
    for (int i = 0; i < 6; ++i) xm[i] = x[i] + 0.5 * p->dt * k1[i];
    orc_car_deriv(p, xm, u, k2);
    for (int i = 0; i < 6; ++i) xn[i] = x[i] + p->dt * k2[i];
}

/* ====================================== track geometry ==================================== */
/* Root of F(s) = (r0 z0 / (s + r0))^2 + (z1 / (s + 1))^2 - 1 by bisection, following Eberly's
 * robust point-to-ellipse distance (Geometric Tools, "Distance from a point to an ellipse..."). */
static double ellipse_root(double r0, double z0, double z1, double g)
{
    double n0 = r0 * z0;
    double s0 = z1 - 1.0;
    double s1 = g < 0.0 ? 0.0 : hypot(n0, z1) - 1.0;
    double s = 0.0;
    for (int it = 0; it < 2000; ++it) {
        s = 0.5 * (s0 + s1);
        if (s == s0 || s == s1) break;
        double ratio0 = n0 / (s + r0), ratio1 = z1 / (s + 1.0);
        double val = ratio0 * ratio0 + ratio1 * ratio1 - 1.0;
        if (val > 0.0) s0 = s; else if (val < 0.0) s1 = s; else break;
    }
    return s;
}

/* Closest point (c0, c1) in the first quadrant of the ellipse with semi-axes e0 >= e1 > 0 to the
 * point (y0, y1) with y0, y1 >= 0. */
static void closest_point_q1(double e0, double e1, double y0, double y1, double* c0, double* c1)
{
    if (y1 > 0.0) {
        if (y0 > 0.0) {
            double z0 = y0 / e0, z1 = y1 / e1;
            double g = z0 * z0 + z1 * z1 - 1.0;
            if (g != 0.0) {
                double r0 = (e0 / e1) * (e0 / e1);
                double sbar = ellipse_root(r0, z0, z1, g);
                *c0 = r0 * y0 / (sbar + r0);
                *c1 = y1 / (sbar + 1.0);
            } else {
                *c0 = y0;
                *c1 = y1;
            }
        } else {
            *c0 = 0.0;
            *c1 = e1;
        }
    } else {
        double numer0 = e0 * y0, denom0 = e0 * e0 - e1 * e1;
        if (numer0 < denom0) {
            double xde0 = numer0 / denom0;
            *c0 = e0 * xde0;
            *c1 = e1 * sqrt(1.0 - xde0 * xde0);
        } else {
            *c0 = e0;
            *c1 = 0.0;
        }
    }
}

/* Signed distance from (X, Y) to the centerline ellipse (X/a)^2 + (Y/b)^2 = 1, positive outside,
 * and the outward unit normal n at the closest point (the gradient of the signed distance).
 * This is the lateral deviation e_y of the track constraints (eqs. 29-33) for a track given as
 * a band of half-width w_T around the ellipse. */
void orc_ellipse_sdf(double a, double b, double X, double Y, double* sd, double n[2])
{
    double ax = fabs(X), ay = fabs(Y);
    double cx, cy;
    if (a >= b) {
        closest_point_q1(a, b, ax, ay, &cx, &cy);
    } else {
        closest_point_q1(b, a, ay, ax, &cy, &cx);
    }
    cx = X < 0.0 ? -cx : cx;
    cy = Y < 0.0 ? -cy : cy;
    double dist = hypot(X - cx, Y - cy);
    double level = (X / a) * (X / a) + (Y / b) * (Y / b);
    *sd = level < 1.0 ? -dist : dist;
    double nx = cx / (a * a), ny = cy / (b * b);
    double nn = hypot(nx, ny);
    n[0] = nx / nn;
    n[1] = ny / nn;
}

/* ================================ belief heuristic and costs ============================== */
/* Belief-space barrier of the track (eq. 33 with eq. 11): e_y = signed distance of the mean
 * position, sigma_y^2 = n^T Sigma_pos n with n = grad e_y (eta in eq. 11), and
 * h = max(w_T - nu sigma_y, 0)^2 - e_y^2.  The clamp at 0 keeps h decreasing in sigma_y once the
 * back-off exceeds the half-width (the literal square is non-monotone there). */
/* Spread of each constraint at a belief (eq. 11, eta the constraint's gradient direction):
 * sig[0] for the track walls (the outward normal of the nearest centerline point), sig[1 + i] for
 * obstacle i (the unit vector from its centre to the mean position; (1, 0) at the centre),
 * sig[5 + i] for half-space constraint i (eta = a_i, its variance a_i^T Sigma a_i held in the
 * record). */
#define SIG_CON 5
static void constraint_sigmas(const orc_params* p, const double mom[ORC_NMOM], double* sig)
{
    double ey, n[2];
    orc_ellipse_sdf(p->ell_a, p->ell_b, mom[0], mom[1], &ey, n);
    double var = n[0] * n[0] * mom[6] + 2.0 * n[0] * n[1] * mom[7] + n[1] * n[1] * mom[8];
    sig[0] = sqrt(var > 0.0 ? var : 0.0);
    for (int i = 0; i < p->n_obs; ++i) {
        double dx = mom[0] - p->obs[3 * i], dy = mom[1] - p->obs[3 * i + 1];
        double d = sqrt(dx * dx + dy * dy);
        double ex = d > 0.0 ? dx / d : 1.0, ey2 = d > 0.0 ? dy / d : 0.0;
        double v = ex * ex * mom[6] + 2.0 * ex * ey2 * mom[7] + ey2 * ey2 * mom[8];
        sig[1 + i] = sqrt(v > 0.0 ? v : 0.0);
    }
    for (int i = 0; i < p->n_con; ++i) {
        double v = mom[9 + i];
        sig[SIG_CON + i] = sqrt(v > 0.0 ? v : 0.0);
    }
}

/* h = min over the constraints (eq. 16) at mean state x with the given spreads: the track walls
 * as eq. 33, h_0 = max(w_T - nu sig_0, 0)^2 - e_y^2, each obstacle in the same form,
 * h_i = max(d_i - nu sig_i, 0)^2 - r_i^2 with d_i the distance to its centre, and each half-space
 * constraint as the heuristic of eq. 13 itself, h_i = -c_i(xbar) - nu sig_i = b_i - a_i^T xbar -
 * nu sig_i (in the units of c_i: a_i and b_i set its weight against the squared-metre terms). */
static double barrier_at(const orc_params* p, double nu, const double x[6], const double* sig)
{
    double X = x[0], Y = x[1];
    double ey, n[2];
    orc_ellipse_sdf(p->ell_a, p->ell_b, X, Y, &ey, n);
    double margin = p->half_width - nu * sig[0];
    if (margin < 0.0) margin = 0.0;
    double h = margin * margin - ey * ey;
    for (int i = 0; i < p->n_obs; ++i) {
        double dx = X - p->obs[3 * i], dy = Y - p->obs[3 * i + 1], r = p->obs[3 * i + 2];
        double m = sqrt(dx * dx + dy * dy) - nu * sig[1 + i];
        if (m < 0.0) m = 0.0;
        double hi = m * m - r * r;
        if (hi < h) h = hi;
    }
    for (int i = 0; i < p->n_con; ++i) {
        const double* a = &p->con_a[6 * i];
        double ax = 0.0;
        for (int j = 0; j < 6; ++j) ax += a[j] * x[j];
        double hi = p->con_b[i] - ax - nu * sig[SIG_CON + i];
        if (hi < h) h = hi;
    }
    return h;
}

double orc_barrier(const orc_params* p, double nu, const double mom[ORC_NMOM])
{
    double sig[SIG_CON + ORC_MAX_CON];
    constraint_sigmas(p, mom, sig);
    return barrier_at(p, nu, mom, sig);
}

/* Running state cost on the mean state (eqs. 27-28, evaluated at xbar as Alg. 1 does):
 * quadratic tracking of the goal speed, lateral deviation and heading error w.r.t. the
 * counter-clockwise tangent (as 2 (1 - cos e_psi), wrap-free), plus the collision penalty
 * C_obs when |e_y| >= w_T. */
double orc_stage_cost(const orc_params* p, const double mom[9])
{
    double ey, n[2];
    orc_ellipse_sdf(p->ell_a, p->ell_b, mom[0], mom[1], &ey, n);
    double tx = -n[1], ty = n[0];
    double cos_epsi = cos(mom[2]) * tx + sin(mom[2]) * ty;
    double dv = mom[3] - p->v_goal;
    double q = p->q_vx * dv * dv + p->q_vy * mom[4] * mom[4] + p->q_r * mom[5] * mom[5] +
               p->q_ey * ey * ey + p->q_epsi * 2.0 * (1.0 - cos_epsi);
    if (fabs(ey) >= p->half_width) q += p->C_obs;
    for (int i = 0; i < p->n_obs; ++i) {
        double dx = mom[0] - p->obs[3 * i], dy = mom[1] - p->obs[3 * i + 1], r = p->obs[3 * i + 2];
        if (dx * dx + dy * dy <= r * r) q += p->C_obs;
    }
    return q;
}

/* ================================== Monte-Carlo moments =================================== */
/* Sample mean (1/M) sum x^n and unbiased covariance 1/(M-1) sum (x^n - xbar)(x^n - xbar)^T of the
 * position block, two-pass.  With a single particle the covariance is defined as 0. */
void orc_moments(const double* particles, int32_t M, double out[9])
{
    for (int i = 0; i < 6; ++i) {
        double acc = 0.0;
        for (int m = 0; m < M; ++m) acc += particles[m * 6 + i];
        out[i] = acc / M;
    }
    double sxx = 0.0, sxy = 0.0, syy = 0.0;
    for (int m = 0; m < M; ++m) {
        double dX = particles[m * 6 + 0] - out[0];
        double dY = particles[m * 6 + 1] - out[1];
        sxx += dX * dX;
        sxy += dX * dY;
        syy += dY * dY;
    }
    if (M > 1) {
        out[6] = sxx / (M - 1);
        out[7] = sxy / (M - 1);
        out[8] = syy / (M - 1);
    } else {
        out[6] = out[7] = out[8] = 0.0;
    }
}

/* Full unbiased covariance 1/(M-1) sum (x^n - xbar)(x^n - xbar)^T of a particle set, two-pass
 * (0 for a single particle): the covariance half of the belief z = [xbar; vec Sigma] (eq. 12). */
void orc_full_cov(const double* particles, int32_t M, double cov[36])
{
    double mean[6];
    for (int i = 0; i < 6; ++i) {
        double acc = 0.0;
        for (int m = 0; m < M; ++m) acc += particles[m * 6 + i];
        mean[i] = acc / M;
    }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double acc = 0.0;
            for (int m = 0; m < M; ++m)
                acc += (particles[m * 6 + i] - mean[i]) * (particles[m * 6 + j] - mean[j]);
            cov[i * 6 + j] = M > 1 ? acc / (double)(M - 1) : 0.0;
        }
}

/* The record's constraint entries from a full covariance: rec[9 + i] = a_i^T Sigma a_i, the
 * variance along the gradient eta_i = a_i of half-space constraint i (eq. 11); 0 beyond n_con. */
void orc_con_spreads(const orc_params* p, const double cov[36], double rec[ORC_NMOM])
{
    for (int i = 0; i < ORC_MAX_CON; ++i) {
        double q = 0.0;
        if (i < p->n_con) {
            const double* a = &p->con_a[6 * i];
            for (int r = 0; r < 6; ++r)
                for (int c = 0; c < 6; ++c) q += a[r] * cov[r * 6 + c] * a[c];
        }
        rec[9 + i] = q;
    }
}

/* ======================================= shield repair ====================================== */
/* One-step DCBF residual of a candidate control at step t: the mean is pushed through the
 * noise-free model and the belief heuristic is re-evaluated with the spread frozen at step t:
 *   r(u) = -h(f(xbar_t, u); sigma_t) + (1 - gamma) h_t.
 * r <= 0 means the linear class-kappa condition (eq. 24) is predicted to hold. */
static double repair_residual(const orc_params* p, double nu, const double mom_t[ORC_NMOM],
                              const double* sig_t, double h_t, const double u[2])
{
    double xn[6];
    orc_model_step(p, mom_t, u, xn);
    double h_next = barrier_at(p, nu, xn, sig_t);
    return -h_next + (1.0 - p->gamma) * h_t;
}

/* Shield repair (the paper describes the S-MPPI repair only as gradient-based minimisation of
 * the DCBF violation and leaves it out of Alg. 1; this is the stated reading): shield_iters
 * damped Gauss-Newton steps toward r = 0,
 *     u <- clip(u - max(r(u), 0) g / (|g|^2 + gmin^2)),   g = dr/du by central differences
 * (step shield_fd).  A step is zero once r <= 0, so a control that already satisfies the
 * condition is returned unchanged; the damping gmin bounds the step where the control has little
 * authority over the next belief, and the map from (u, belief) to the repaired control is
 * continuous. */
void orc_repair(const orc_params* p, double nu, const double mom_t[ORC_NMOM], double u[2])
{
    if (p->shield_iters <= 0) return;
    double sigma_t[SIG_CON + ORC_MAX_CON];
    constraint_sigmas(p, mom_t, sigma_t);
    double h_t = orc_barrier(p, nu, mom_t);
    double fd = p->shield_fd;
    for (int it = 0; it < p->shield_iters; ++it) {
        double r0 = repair_residual(p, nu, mom_t, sigma_t, h_t, u);
        if (!(r0 > 0.0)) break;
        double g[2];
        for (int j = 0; j < 2; ++j) {
            double up[2] = {u[0], u[1]}, um[2] = {u[0], u[1]};
            up[j] += fd;
            um[j] -= fd;
            g[j] = (repair_residual(p, nu, mom_t, sigma_t, h_t, up) -
                    repair_residual(p, nu, mom_t, sigma_t, h_t, um)) / (2.0 * fd);
        }
        double denom = g[0] * g[0] + g[1] * g[1] + p->shield_gmin * p->shield_gmin;
        u[0] = clampd(u[0] - r0 * g[0] / denom, -p->steer_max, p->steer_max);
        u[1] = clampd(u[1] - r0 * g[1] / denom, -p->accel_max, p->accel_max);
    }
}

/* ===================================== trajectory cost ====================================== */
/* Trajectory cost of one sample from its belief trajectory (moments at t = 0..T) and its controls
 * (Alg. 1): S = sum_{t<T} [q(xbar_t) + gamma_u v_t^T Sigma_eps^-1 u_t + C_safe(z_t)]
 *             + phi(xbar_T) + C_safe(z_T),
 * with C_safe(z_t) = C max(-h_t + (1 - gamma) h_{t-1}, 0) (eq. 25) and C_safe(z_0) = 0 (the
 * convention z_0^(2) = z_0^(1)).  phi = phi_scale * q.  A zero noise std gives a zero weight. */
double orc_score(const orc_params* p, double nu, const double* mom, const double* u,
                 const double* v)
{
    int T = p->T;
    double inv_var[2];
    for (int j = 0; j < 2; ++j)
        inv_var[j] = p->sigma_eps[j] > 0.0 ? 1.0 / (p->sigma_eps[j] * p->sigma_eps[j]) : 0.0;
    double S = 0.0;
    double h_prev = orc_barrier(p, nu, &mom[0]);
    for (int t = 0; t < T; ++t) {
        const double* mt = &mom[(size_t)t * ORC_NMOM];
        double h_t = orc_barrier(p, nu, mt);
        double c_safe = 0.0;
        if (t > 0) {
            double viol = -h_t + (1.0 - p->gamma) * h_prev;
            c_safe = p->C_cbf * (viol > 0.0 ? viol : 0.0);
        }
        double ctrl = p->gamma_u * (v[t * 2 + 0] * inv_var[0] * u[t * 2 + 0] +
                                    v[t * 2 + 1] * inv_var[1] * u[t * 2 + 1]);
        S += orc_stage_cost(p, mt) + ctrl + c_safe;
        h_prev = h_t;
    }
    const double* mT = &mom[(size_t)T * ORC_NMOM];
    double h_T = orc_barrier(p, nu, mT);
    double viol = -h_T + (1.0 - p->gamma) * h_prev;
    S += p->phi_scale * orc_stage_cost(p, mT) + p->C_cbf * (viol > 0.0 ? viol : 0.0);
    return S;
}

/* ======================================== one rollout ======================================== */
/* Initial particles x^n_0 = xbar_0 + L_0 xi^n (tag 2) and the t = 0 belief record (the given
 * estimate, Alg. 1 initialisation). */
static void init_particles(const orc_params* p, uint32_t s, int32_t k, const double x0[6],
                           const double* Sigma0, const double* L0, double* part, double* mom0)
{
    uint32_t ctr[4];
    double z[4];
    for (int m = 0; m < p->M; ++m) {
        double xi[6] = {0, 0, 0, 0, 0, 0};
        if (L0) {
            for (uint32_t blk = 0; blk < 2; ++blk) {
                rng_counter(blk, (uint32_t)m, (uint32_t)k, 2u, s, ctr);
                orc_normals(p->seed, ctr, z);
                xi[blk * 3 + 0] = z[0];
                xi[blk * 3 + 1] = z[1];
                xi[blk * 3 + 2] = z[2];
            }
        }
        for (int i = 0; i < 6; ++i) {
            double acc = x0[i];
            for (int j = 0; j < 6; ++j) acc += (L0 ? L0[i * 6 + j] : 0.0) * xi[j];
            part[m * 6 + i] = acc;
        }
    }
    for (int i = 0; i < 6; ++i) mom0[i] = x0[i];
    mom0[6] = Sigma0 ? Sigma0[0] : 0.0;
    mom0[7] = Sigma0 ? Sigma0[1] : 0.0;
    mom0[8] = Sigma0 ? Sigma0[7] : 0.0;
    double cov0[36];
    for (int i = 0; i < 36; ++i) cov0[i] = Sigma0 ? Sigma0[i] : 0.0;
    orc_con_spreads(p, cov0, mom0);
}

void orc_chol_psd6(const double* A, double* L)
{
    memset(L, 0, sizeof(double) * 36);
    for (int j = 0; j < 6; ++j) {
        double d = A[j * 6 + j];
        for (int q = 0; q < j; ++q) d -= L[j * 6 + q] * L[j * 6 + q];
        if (d <= 1e-10 * A[j * 6 + j] + 1e-24) continue;
        double ljj = sqrt(d);
        L[j * 6 + j] = ljj;
        for (int i = j + 1; i < 6; ++i) {
            double acc = A[i * 6 + j];
            for (int q = 0; q < j; ++q) acc -= L[i * 6 + q] * L[j * 6 + q];
            L[i * 6 + j] = acc / ljj;
        }
    }
}

/* Gaussian re-sampling of Alg. 2 as printed: the particles of step t are redrawn as
 * x^n_t = xbar_t + L_t xi^n with xbar_t and the unbiased full 6x6 covariance Sigma_t of the
 * current set (two-pass; Sigma := 0 for M = 1), L_t its semi-definite factor, and xi^n six
 * standard normals from tags 4 and 5 with counter (t, n, k). */
static void resample_particles(const orc_params* p, uint32_t s, int32_t k, int t, double* part)
{
    int M = p->M;
    double mean[6] = {0, 0, 0, 0, 0, 0}, cov[36], L[36];
    for (int m = 0; m < M; ++m)
        for (int i = 0; i < 6; ++i) mean[i] += part[m * 6 + i];
    for (int i = 0; i < 6; ++i) mean[i] /= (double)M;
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double acc = 0.0;
            for (int m = 0; m < M; ++m)
                acc += (part[m * 6 + i] - mean[i]) * (part[m * 6 + j] - mean[j]);
            cov[i * 6 + j] = M > 1 ? acc / (double)(M - 1) : 0.0;
        }
    orc_chol_psd6(cov, L);
    uint32_t ctr[4];
    double z[4];
    for (int m = 0; m < M; ++m) {
        double xi[6];
        for (uint32_t blk = 0; blk < 2; ++blk) {
            rng_counter((uint32_t)t, (uint32_t)m, (uint32_t)k, 4u + blk, s, ctr);
            orc_normals(p->seed, ctr, z);
            xi[blk * 3 + 0] = z[0];
            xi[blk * 3 + 1] = z[1];
            xi[blk * 3 + 2] = z[2];
        }
        for (int i = 0; i < 6; ++i) {
            double acc = mean[i];
            for (int j = 0; j <= i; ++j) acc += L[i * 6 + j] * xi[j];
            part[m * 6 + i] = acc;
        }
    }
}

/* Sigma-point propagation (the unscented/cubature alternative to Monte Carlo): the belief
 * (mean, full 6x6 covariance) is represented by the 12 points mean +- sqrt(6) L e_i (L the
 * semi-definite factor, equal weights 1/12), each propagated through the noise-free model; the
 * new belief is their weighted mean and covariance plus the disturbance covariance
 * Q diag(0, 0, 0, sigma_w^2) scaled by the points' mean of (1 + kappa |vx|)^2. */
static void sigma_points(const double mean[6], const double cov[36], double* part)
{
    double L[36];
    orc_chol_psd6(cov, L);
    const double r = sqrt(6.0);
    for (int i = 0; i < 6; ++i)
        for (int a = 0; a < 6; ++a) {
            part[i * 6 + a] = mean[a] + r * L[a * 6 + i];
            part[(6 + i) * 6 + a] = mean[a] - r * L[a * 6 + i];
        }
}

static void sigma_step(const orc_params* p, const double u[2], double* part, double* nxt,
                       double* mom_next, double* cov_next)
{
    double mean[6] = {0, 0, 0, 0, 0, 0}, q = 0.0;
    for (int i = 0; i < 12; ++i) {
        double sc = 1.0 + p->sigma_w_speed * fabs(part[i * 6 + 3]);
        q += sc * sc / 12.0;
        orc_model_step(p, &part[i * 6], u, &nxt[i * 6]);
    }
    for (int i = 0; i < 12; ++i)
        for (int a = 0; a < 6; ++a) mean[a] += nxt[i * 6 + a] / 12.0;
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) {
            double acc = 0.0;
            for (int i = 0; i < 12; ++i)
                acc += (nxt[i * 6 + a] - mean[a]) * (nxt[i * 6 + b] - mean[b]);
            cov_next[a * 6 + b] = acc / 12.0;
        }
    for (int a = 0; a < 3; ++a) cov_next[(3 + a) * 6 + 3 + a] += p->sigma_w[a] * p->sigma_w[a] * q;
    for (int a = 0; a < 6; ++a) mom_next[a] = mean[a];
    mom_next[6] = cov_next[0];
    mom_next[7] = cov_next[1];
    mom_next[8] = cov_next[7];
    orc_con_spreads(p, cov_next, mom_next);
    sigma_points(mean, cov_next, part);
}

/* The three standard normals of the disturbance of particle m at step t (tag 1).  Particles come
 * in quads: quad q = m / 4 owns the three Philox blocks with counter words (t, 3q + b, k) for
 * b = 0, 1, 2, whose twelve normals (block b gives normals 4b .. 4b+3) are dealt out three per
 * particle in order: particle 4q + i takes normals 3i, 3i + 1 and 3i + 2.  Every normal of a block
 * is used. */
void orc_disturbance_normals(uint64_t seed, uint32_t s, uint32_t k, uint32_t t, uint32_t m,
                             double w[3])
{
    uint32_t q = m / 4u, i = m % 4u;
    double z12[12];
    for (uint32_t b = 0; b < 3; ++b) {
        uint32_t ctr[4];
        rng_counter(t, 3u * q + b, k, 1u, s, ctr);
        orc_normals(seed, ctr, &z12[4 * b]);
    }
    for (int c = 0; c < 3; ++c) w[c] = z12[3 * i + c];
}

/* One step of Alg. 2 with persistent particles: x^n_{t+1} = f(x^n_t, u_t) + [0,0,0, w^n_t]
 * (w from tag 1, orc_disturbance_normals), then the moments of the new particle set.  The
 * disturbance may depend on the state (p(w|x)): its std is sigma_w (1 + kappa |vx^n_t|); with
 * common random numbers every sample draws it with counter word k = 0. */
static void propagate_step(const orc_params* p, uint32_t s, int32_t k, int t, const double u[2],
                           double* part, double* nxt, double* mom_next)
{
    double z[3];
    int M = p->M;
    uint32_t kw = p->crn ? 0u : (uint32_t)k;
    for (int m = 0; m < M; ++m) {
        double scale = 1.0 + p->sigma_w_speed * fabs(part[m * 6 + 3]);
        orc_model_step(p, &part[m * 6], u, &nxt[m * 6]);
        orc_disturbance_normals(p->seed, s, kw, (uint32_t)t, (uint32_t)m, z);
        nxt[m * 6 + 3] += p->sigma_w[0] * scale * z[0];
        nxt[m * 6 + 4] += p->sigma_w[1] * scale * z[1];
        nxt[m * 6 + 5] += p->sigma_w[2] * scale * z[2];
    }
    memcpy(part, nxt, sizeof(double) * 6 * (size_t)M);
    orc_moments(part, M, mom_next);
    double cov[36];
    orc_full_cov(part, M, cov);
    orc_con_spreads(p, cov, mom_next);
}

/* Belief at t = 0: Monte-Carlo particles (init_particles), or the sigma points of (x0, Sigma0). */
static void init_belief(const orc_params* p, uint32_t s, int32_t k, const double x0[6],
                        const double* Sigma0, const double* L0, double* part, double* mom0,
                        double* cov)
{
    init_particles(p, s, k, x0, Sigma0, L0, part, mom0);
    if (p->belief == 2) {
        for (int i = 0; i < 36; ++i) cov[i] = Sigma0 ? Sigma0[i] : 0.0;
        sigma_points(x0, cov, part);
    }
}

/* One step of the belief recursion in the selected reading (persistent particles, re-sampling
 * or sigma points). */
static void advance_belief(const orc_params* p, uint32_t s, int32_t k, int t, const double u[2],
                           double* part, double* nxt, double* mom_next, double* cov)
{
    if (p->belief == 2) {
        sigma_step(p, u, part, nxt, mom_next, cov);
        return;
    }
    if (p->belief == 1 && t > 0) resample_particles(p, s, k, t, part);
    propagate_step(p, s, k, t, u, part, nxt, mom_next);
}

/* Sample k of Alg. 1: draw eps_{k,t}, form u = clip(v + eps), optionally repair it, propagate the
 * M persistent particles x^n_{t+1} = f(x^n_t, u_t) + w^n_t through the model (the particle
 * recursion stated with the Monte-Carlo covariance), record the moments, and score. */
double orc_rollout(const orc_params* p, double nu, uint32_t s, int32_t k, const double x0[6],
                   const double* Sigma0, const double* L0, const double* v, double* u_out,
                   double* mom_out)
{
    int M = p->M, T = p->T;
    size_t np = (size_t)(M > 12 ? M : 12);   /* sigma points use 12 */
    double* part = (double*)malloc(sizeof(double) * 6 * np);
    double* nxt = (double*)malloc(sizeof(double) * 6 * np);
    uint32_t ctr[4];
    double z[4], cov[36];
    init_belief(p, s, k, x0, Sigma0, L0, part, mom_out, cov);
    for (int t = 0; t < T; ++t) {
        rng_counter((uint32_t)t, 0u, (uint32_t)k, 0u, s, ctr);
        orc_normals(p->seed, ctr, z);
        double u[2];
        u[0] = clampd(v[t * 2 + 0] + p->sigma_eps[0] * z[0], -p->steer_max, p->steer_max);
        u[1] = clampd(v[t * 2 + 1] + p->sigma_eps[1] * z[1], -p->accel_max, p->accel_max);
        orc_repair(p, nu, &mom_out[(size_t)t * ORC_NMOM], u);
        u_out[t * 2 + 0] = u[0];
        u_out[t * 2 + 1] = u[1];
        advance_belief(p, s, k, t, u, part, nxt, &mom_out[(size_t)(t + 1) * ORC_NMOM], cov);
    }
    free(part);
    free(nxt);
    return orc_score(p, nu, mom_out, u_out, v);
}

/* Belief trajectory of sample k for a given control sequence u [T][2] (no sampling, no repair):
 * the propagation half of a rollout, used to check the particle propagation on its own. */
void orc_propagate(const orc_params* p, uint32_t s, int32_t k, const double x0[6],
                   const double* Sigma0, const double* L0, const double* u, double* mom_out)
{
    int M = p->M, T = p->T;
    size_t np = (size_t)(M > 12 ? M : 12);   /* sigma points use 12 */
    double* part = (double*)malloc(sizeof(double) * 6 * np);
    double* nxt = (double*)malloc(sizeof(double) * 6 * np);
    double cov[36];
    init_belief(p, s, k, x0, Sigma0, L0, part, mom_out, cov);
    for (int t = 0; t < T; ++t)
        advance_belief(p, s, k, t, &u[t * 2], part, nxt, &mom_out[(size_t)(t + 1) * ORC_NMOM],
                       cov);
    free(part);
    free(nxt);
}

/* ======================================= MPPI update ======================================== */
/* beta = min_k S_k, w_k = exp(-(S_k - beta) / lambda) (eq. 7), and the update of eq. 6 written as
 * v+ = v + sum_k w_k (u_k - v) / sum_k w_k (algebraically equal, better conditioned).  Non-finite
 * costs get weight 0; if none is finite, v is left unchanged and 1 is returned.
 * stats = {beta, Z = sum w, effective sample size Z^2 / sum w^2, number of finite costs}. */
int32_t orc_update(const orc_params* p, const double* S, const double* u, double* v,
                   double stats[4])
{
    int K = p->K, T = p->T;
    double beta = INFINITY;
    int n_finite = 0;
    for (int k = 0; k < K; ++k) {
        if (isfinite(S[k])) {
            ++n_finite;
            if (S[k] < beta) beta = S[k];
        }
    }
    if (n_finite == 0) return 1;
    double* w = (double*)malloc(sizeof(double) * (size_t)K);
    double Z = 0.0, W2 = 0.0;
    for (int k = 0; k < K; ++k) {
        w[k] = isfinite(S[k]) ? exp(-(S[k] - beta) / p->lambda) : 0.0;
        Z += w[k];
        W2 += w[k] * w[k];
    }
    for (int t = 0; t < T; ++t) {
        for (int j = 0; j < 2; ++j) {
            double acc = 0.0;
            for (int k = 0; k < K; ++k)
                acc += w[k] * (u[((size_t)k * T + t) * 2 + j] - v[t * 2 + j]);
            v[t * 2 + j] += acc / Z;
        }
    }
    free(w);
    if (stats) {
        stats[0] = beta;
        stats[1] = Z;
        stats[2] = Z * Z / W2;
        stats[3] = n_finite;
    }
    return 0;
}

/* =========================================== solve =========================================== */
/* Lower Cholesky factor of a symmetric positive semi-definite 6x6 matrix (a zero pivot gives a
 * zero column). */
static void cholesky6(const double* A, double* L)
{
    memset(L, 0, sizeof(double) * 36);
    for (int j = 0; j < 6; ++j) {
        double d = A[j * 6 + j];
        for (int q = 0; q < j; ++q) d -= L[j * 6 + q] * L[j * 6 + q];
        if (d <= 0.0) continue;
        double ljj = sqrt(d);
        L[j * 6 + j] = ljj;
        for (int i = j + 1; i < 6; ++i) {
            double acc = A[i * 6 + j];
            for (int q = 0; q < j; ++q) acc -= L[i * 6 + q] * L[j * 6 + q];
            L[i * 6 + j] = acc / ljj;
        }
    }
}

/* Repair of the updated sequence from the state estimate (the local repair of v+ that Alg. 1
 * carries between the update and the executed command): one more rollout from (xbar_0, Sigma_0)
 * whose control at step t is clip(v+_t), repaired against that rollout's belief at t exactly as
 * a sampled control is (orc_repair), then propagated; the repaired controls form v_safe.  The
 * rollout's particles draw their disturbance and initial spread from a stream of their own: the
 * Philox key of seed ^ ORC_LOCAL_REPAIR_KEY with sample word 0 and the solve's index s.
 * mom_out [T+1][ORC_NMOM] may be NULL. */
#define ORC_LOCAL_REPAIR_KEY 0x5DEECE66DA3B9F1Bull

void orc_local_repair(const orc_params* p, uint32_t s, const double x0[6], const double* Sigma0,
                      const double* v_plus, double* v_safe, double* mom_out)
{
    orc_params q = *p;
    q.seed = p->seed ^ ORC_LOCAL_REPAIR_KEY;
    q.sigma_eps[0] = 0.0;
    q.sigma_eps[1] = 0.0;
    double nu = orc_backoff(p->delta, p->backoff);
    double L0[36];
    int use_spread = 0;
    if (Sigma0) {
        cholesky6(Sigma0, L0);
        for (int i = 0; i < 36; ++i) use_spread |= (Sigma0[i] != 0.0);
    }
    double* mom = mom_out ? mom_out
                          : (double*)malloc(sizeof(double) * (size_t)(p->T + 1) * ORC_NMOM);
    (void)orc_rollout(&q, nu, s, 0, x0, Sigma0, use_spread ? L0 : NULL, v_plus, v_safe, mom);
    if (!mom_out) free(mom);
}

typedef struct {
    const orc_params* p;
    double nu;
    uint32_t s;
    const double* x0;
    const double* Sigma0;
    const double* L0;
    const double* v;
    double* u;
    double* mom;
    double* S;
    int k_begin, k_end;
} rollout_job;

static void* rollout_worker(void* arg)
{
    rollout_job* job = (rollout_job*)arg;
    const orc_params* p = job->p;
    size_t T = (size_t)p->T;
    for (int k = job->k_begin; k < job->k_end; ++k) {
        double* mom_k = &job->mom[(size_t)k * (T + 1) * ORC_NMOM];
        double* u_k = &job->u[(size_t)k * T * 2];
        job->S[k] = orc_rollout(p, job->nu, job->s, k, job->x0, job->Sigma0, job->L0, job->v,
                                u_k, mom_k);
    }
    return NULL;
}

/* One BSS-MPPI solve (Alg. 1, one pass of the while-loop body): all K rollouts, then the
 * update of v in place, then (local_repair 1 or 2) the repair of the updated sequence from the
 * estimate; with local_repair = 2 the sampled controls are not repaired.  Sigma0 (6x6,
 * row-major) may be NULL for a known initial state.
 * u_out [K][T][2], mom_out [K][T+1][ORC_NMOM] and S_out [K] may be NULL.  Work is split over K
 * across nthreads threads; results do not depend on the split. Returns 0, or 1 when no cost is
 * finite. */
int32_t orc_solve(const orc_params* p, uint32_t s, const double x0[6], const double* Sigma0,
                  double* v, double* u_out, double* mom_out, double* S_out, double stats[4],
                  int32_t nthreads)
{
    int K = p->K, T = p->T;
    double nu = orc_backoff(p->delta, p->backoff);
    double L0[36];
    int use_spread = 0;
    if (Sigma0) {
        cholesky6(Sigma0, L0);
        for (int i = 0; i < 36; ++i) use_spread |= (Sigma0[i] != 0.0);
    }
    double* u = u_out ? u_out : (double*)malloc(sizeof(double) * (size_t)K * T * 2);
    double* mom = mom_out ? mom_out
                          : (double*)malloc(sizeof(double) * (size_t)K * (T + 1) * ORC_NMOM);
    double* S = S_out ? S_out : (double*)malloc(sizeof(double) * (size_t)K);

    orc_params ps = *p;   /* the samples' settings */
    if (p->local_repair == 2) ps.shield_iters = 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > K) nthreads = K;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    rollout_job* jobs = (rollout_job*)malloc(sizeof(rollout_job) * (size_t)nthreads);
    for (int i = 0; i < nthreads; ++i) {
        rollout_job j = {&ps, nu, s, x0, Sigma0, use_spread ? L0 : NULL, v,
                         u, mom, S, (int)((long)K * i / nthreads),
                         (int)((long)K * (i + 1) / nthreads)};
        jobs[i] = j;
        if (nthreads == 1) rollout_worker(&jobs[i]);
        else pthread_create(&th[i], NULL, rollout_worker, &jobs[i]);
    }
    if (nthreads > 1)
        for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
    free(th);
    free(jobs);

    int32_t rc = orc_update(p, S, u, v, stats);
    if (p->local_repair) {
        double* v_safe = (double*)malloc(sizeof(double) * (size_t)T * 2);
        orc_local_repair(p, s, x0, Sigma0, v, v_safe, NULL);
        memcpy(v, v_safe, sizeof(double) * (size_t)T * 2);
        free(v_safe);
    }
    if (!u_out) free(u);
    if (!mom_out) free(mom);
    if (!S_out) free(S);
    return rc;
}

/* Warm start for the next control period: shift the sequence left by one step and repeat the
 * last element (Alg. 1 reuses v; the shift is the usual receding-horizon warm start). */
void orc_step_shift(int32_t T, double* v)
{
    for (int t = 0; t + 1 < T; ++t) {
        v[t * 2 + 0] = v[(t + 1) * 2 + 0];
        v[t * 2 + 1] = v[(t + 1) * 2 + 1];
    }
}
