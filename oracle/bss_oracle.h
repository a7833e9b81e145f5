/*
 * bss_oracle.h -- plain FP64 CPU oracle for belief-space stochastic MPPI (BSS-MPPI).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct reference that the
 * GPU path is checked against.  Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it; the product path never calls it and shares no code with it.
 *
 * Everything is double precision.  Paper references are to "Chance-Constrained
 * Information-Theoretic Stochastic MPC with Safety Shielding" (Yin, Tsiotras, Berntorp,
 * arXiv 2408.00494): eq. numbers follow the order of the paper's displayed equations,
 * Alg. 1 is the BSS-MPPI algorithm and Alg. 2 the Monte-Carlo mean/covariance propagation.
 */
#ifndef BSS_ORACLE_H
#define BSS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Problem description.  Field meanings:
 *  car (6 states X, Y, psi, vx, vy, r; 2 controls steer [rad], accel [m/s^2]):
 *    m [kg], Iz [kg m^2], lf, lr [m], Cf, Cr [N/rad], mu, g, v_min [m/s] (slip-angle floor), dt [s]
 *  steer_max, accel_max: symmetric control box
 *  sigma_eps: control-noise std (u ~ N(v, Sigma_eps), Sigma_eps diagonal)
 *  sigma_w:   per-step disturbance std on (vx, vy, r)
 *  K control samples, M disturbance particles per sample, T horizon steps
 *  delta: per-wall violation probability; gamma: linear class-kappa rate (beta in the paper's
 *    linear DCBF condition); backoff: 0 Gaussian nu = sqrt(2) erfinv(1-2 delta), 1 Cantelli
 *  lambda: MPPI temperature; gamma_u: control-cost weight of the trajectory cost
 *  v_goal, q_*: tracking weights; C_cbf: safety-violation weight C; C_obs: collision penalty;
 *  phi_scale: terminal cost = phi_scale * running cost
 *  ell_a, ell_b: centerline ellipse semi-axes [m]; half_width: w_T [m]
 *  shield_iters, shield_gmin, shield_fd: shield repair (0 iterations = no repair), its
 *    damping and its finite-difference step
 *  seed: Philox key
 *  model: 0 = car with explicit-midpoint RK2, 1 = linear test model x+ = A x + B u (+ noise)
 *  n_con, con_a, con_b: up to four half-space constraints on the whole state,
 *    c_i(x) = a_i^T x - b_i <= 0 with a_i = con_a[6i..6i+5] over (X, Y, psi, vx, vy, r), each a
 *    further chance constraint with gradient eta_i = a_i and heuristic
 *    h_i = b_i - a_i^T xbar - nu sqrt(a_i^T Sigma a_i) over the full 6x6 covariance Sigma
 */
typedef struct orc_params {
    double m, Iz, lf, lr, Cf, Cr, mu, g, v_min, dt;
    double steer_max, accel_max;
    double sigma_eps[2];
    double sigma_w[3];
    int32_t K, M, T;
    double delta, gamma;
    int32_t backoff;
    double lambda, gamma_u, v_goal, q_vx, q_vy, q_r, q_ey, q_epsi, C_cbf, C_obs, phi_scale;
    double ell_a, ell_b, half_width;
    int32_t shield_iters;
    double shield_gmin, shield_fd;
    uint64_t seed;
    int32_t belief;       /* 0 persistent particles, 1 Gaussian re-sampling every step,
                             2 sigma points (12-point cubature set, M = 12) */
    int32_t crn;          /* 1: every sample draws the same disturbances (counter word k = 0) */
    double sigma_w_speed; /* kappa: disturbance std sigma_w (1 + kappa |vx|) at the step's state */
    int32_t n_obs;        /* circular obstacles (0..4), each a further chance constraint */
    double obs[12];       /* obstacle i: centre (obs[3i], obs[3i+1]), radius obs[3i+2] */
    int32_t local_repair; /* repair of the updated sequence from the estimate (the local repair
                             of v+ in Alg. 1): 0 off, 1 after the update and in every sample,
                             2 after the update only */
    int32_t model;
    double lin_A[36];
    double lin_B[12];
    int32_t n_con;        /* half-space state constraints (0..4) */
    double con_a[24];     /* constraint i: a_i = con_a[6i..6i+5] */
    double con_b[4];      /* constraint i: bound b_i */
    /* vehicle: 0 = the 6-state car above; 1 = the paper's 8-state single-track vehicle with wheel
     * speeds in the road-aligned frame (bss_oracle8.c), x = [vX, vY, r, wF, wR, epsi, eY, s],
     * u = [steer, throttle], reusing m, Iz, lf, lr, mu, g, v_min, dt, the control box
     * (accel_max bounds the throttle), the noise, the weights and half_width */
    int32_t vehicle;
    double Rw, Iw, T_max;              /* wheel radius [m], drive-line inertia per axle [kg m^2],
                                          rear drive torque at full throttle [N m] */
    double pac_B, pac_C, pac_D, pac_E; /* magic-formula coefficients (pure slip) */
    double track_len, kappa_amp;       /* centerline curvature (2 pi / L)(1 + a sin(4 pi s / L)) */
    int32_t n_sub;                     /* explicit-midpoint substeps per control period */
} orc_params;

#define ORC_MAX_CON 4

/* Layout of one belief record (13 doubles): mean X, Y, psi, vx, vy, r, then the position
 * covariance Sxx, Sxy, Syy, then a_i^T Sigma a_i for the half-space constraints i < n_con (0 in
 * the unused entries).  The belief z = [xbar; vec Sigma] of eq. 12 enters the heuristic only
 * through these projections of Sigma, so only they are kept; the last four come from the full
 * 6x6 covariance. */
#define ORC_NMOM 13

/* ---- random numbers: Philox4x32-10 (Salmon et al., SC'11) and Box-Muller --------------- */
void   orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_uniform(uint32_t r);
void   orc_normals(uint64_t seed, const uint32_t ctr[4], double z[4]);
void   orc_philox_many(const uint32_t* ctr, const uint32_t key[2], uint32_t* out, int64_t n);
void   orc_normals_many(uint64_t seed, const uint32_t* ctr, double* z, int64_t n);
/* Disturbance normals w[3] of particle m at step t of sample word k under solve index s: particle
 * quad q = m / 4 owns the blocks with counter (t, 3q + b, k, (1 << 28) | s), b = 0..2, whose twelve
 * normals are dealt out three per particle (particle 4q + i takes normals 3i .. 3i + 2). */
void   orc_disturbance_normals(uint64_t seed, uint32_t s, uint32_t k, uint32_t t, uint32_t m,
                               double w[3]);

/* Lower factor L of a symmetric positive semi-definite 6x6 matrix with L L^T = A, by columns; a
 * pivot d <= 1e-10 A_jj + 1e-24 counts as zero and leaves its column zero (so variances at the
 * rounding level of an exactly degenerate set are not amplified). */
void orc_chol_psd6(const double* A, double* L);

/* ---- back-off coefficient (Remark 1) ---------------------------------------------------- */
double orc_backoff(double delta, int32_t backoff);

/* ---- dynamics ----------------------------------------------------------------------------- */
void orc_car_deriv(const orc_params* p, const double x[6], const double u[2], double dx[6]);
void orc_model_step(const orc_params* p, const double x[6], const double u[2], double xn[6]);

/* ---- track geometry and belief heuristic ------------------------------------------------ */
void   orc_ellipse_sdf(double a, double b, double X, double Y, double* sd, double n[2]);
double orc_barrier(const orc_params* p, double nu, const double mom[ORC_NMOM]);
double orc_stage_cost(const orc_params* p, const double mom[9]);

/* ---- Monte-Carlo moments (Alg. 2) --------------------------------------------------------- */
void orc_moments(const double* particles, int32_t M, double out[9]);
void orc_full_cov(const double* particles, int32_t M, double cov[36]);
void orc_con_spreads(const orc_params* p, const double cov[36], double rec[ORC_NMOM]);

/* ---- shield repair of one control ------------------------------------------------------- */
void orc_repair(const orc_params* p, double nu, const double mom_t[ORC_NMOM], double u[2]);

/* ---- one sample's rollout and its cost ---------------------------------------------------- */
double orc_score(const orc_params* p, double nu, const double* mom, const double* u,
                 const double* v);
double orc_rollout(const orc_params* p, double nu, uint32_t s, int32_t k, const double x0[6],
                   const double* Sigma0, const double* L0, const double* v, double* u_out,
                   double* mom_out);

void orc_propagate(const orc_params* p, uint32_t s, int32_t k, const double x0[6],
                   const double* Sigma0, const double* L0, const double* u, double* mom_out);

/* ---- MPPI update (eqs. 6-7) ---------------------------------------------------------------- */
int32_t orc_update(const orc_params* p, const double* S, const double* u, double* v,
                   double stats[4]);

/* ---- one full solve -------------------------------------------------------------------------- */
int32_t orc_solve(const orc_params* p, uint32_t s, const double x0[6], const double* Sigma0,
                  double* v, double* u_out, double* mom_out, double* S_out, double stats[4],
                  int32_t nthreads);

/* repair of the updated sequence from the estimate (local_repair; v_safe [T][2], mom_out
 * [T+1][ORC_NMOM] or NULL) */
void orc_local_repair(const orc_params* p, uint32_t s, const double x0[6], const double* Sigma0,
                      const double* v_plus, double* v_safe, double* mom_out);

void orc_step_shift(int32_t T, double* v);

/* ---- the 8-state vehicle (vehicle = 1; bss_oracle8.c) ---------------------------------------
 * Records hold 9 doubles: the means of the 8 states, then the unbiased variance of eY. */
#define ORC8_NX 8
#define ORC8_NREC 9
double orc8_magic(const orc_params* p, double z);
void   orc8_tire(const orc_params* p, double Fz, double slip, double alpha, double F[2]);
double orc8_kappa(const orc_params* p, double s);
void   orc8_deriv(const orc_params* p, const double x[8], const double u[2], double dx[8]);
void   orc8_step(const orc_params* p, const double x[8], const double u[2], double xn[8]);
void   orc8_moments(const double* particles, int32_t M, double rec[9]);
double orc8_barrier(const orc_params* p, double nu, const double rec[9]);
double orc8_stage_cost(const orc_params* p, const double rec[9]);
void   orc8_repair(const orc_params* p, double nu, const double rec_t[9], double u[2]);
double orc8_score(const orc_params* p, double nu, const double* rec, const double* u,
                  const double* v);
int32_t orc8_solve(const orc_params* p, uint32_t s, const double x0[8], double* v, double* u_out,
                   double* rec_out, double* S_out, double stats[4], int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
