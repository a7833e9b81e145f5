/*
 * bssmppi.h -- C ABI of libbssmppi: belief-space stochastic MPPI (BSS-MPPI) on AMD MI355X (gfx950).
 *
 * Method: Yin, Tsiotras, Berntorp, "Chance-Constrained Information-Theoretic Stochastic MPC with
 * Safety Shielding" (arXiv 2408.00494).  One solve is one pass of the body of the paper's Alg. 1:
 * K control sequences u_k ~ N(v, Sigma_eps) are sampled (clipped to the control box, optionally
 * shield-repaired); each is pushed through M Monte-Carlo disturbance particles of the dynamics
 * over T steps (Alg. 2, persistent particles); the per-step particle mean and position covariance
 * (the belief z = [xbar; Sigma]) are scored with the tracking cost, the collision indicator and the
 * safety-violation cost C_safe of the belief-space DCBF (eqs. 11, 13, 24-26, 33); the K costs are
 * folded into the MPPI update v+ = sum_k w_k u_k / sum_k w_k, w_k = exp(-(S_k - min S)/lambda)
 * (eqs. 6-8).  The dynamics is a single-track car with linear tires; the track is a band of
 * half-width w_T around an ellipse.
 *
 * Precision: particles are propagated in single precision; moments, scores, the shield repair and
 * the update are accumulated in double precision on the device.
 *
 * Conventions for every call:
 *   - Return values are bss_status codes; on failure a message is available from
 *     bss_last_error() (thread-local, valid until the next failing call on that thread).
 *   - The library never aborts and never prints.
 *   - "device" pointers are HIP device addresses on the context's device; "host" pointers are
 *     ordinary host memory.  Ownership stays with the caller unless stated otherwise.
 *   - A context is not thread-safe; distinct contexts may be used from different threads.
 */
#ifndef BSSMPPI_H
#define BSSMPPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bss_status {
    BSS_OK = 0,
    BSS_E_INVAL = 1,    /* invalid argument or parameter set                          */
    BSS_E_NOMEM = 2,    /* device or host allocation failed                           */
    BSS_E_DEVICE = 3,   /* a HIP runtime call or kernel launch failed                 */
    BSS_E_STATE = 4,    /* call not valid in the context's current state              */
    BSS_E_NUMERIC = 5   /* no sample had a finite cost; the mean controls were kept   */
} bss_status;

/* Problem description (copied at bss_create; the caller keeps ownership).
 * Dynamics (single-track car, x = [X, Y, psi, vx, vy, r], u = [steer rad, accel m/s^2]):
 *   slip angles a_f = steer - atan((vy + lf r)/max(vx, v_min)), a_r = -atan((vy - lr r)/max(vx, v_min));
 *   lateral forces F = C a clipped to +-mu m g (axle load share); explicit midpoint (RK2) step of
 *   length dt with zero-order hold on u; the disturbance w ~ N(0, diag(sigma_w^2)) is added to
 *   (vx, vy, r) after each step (the disturbed system of eq. 5b).
 * Sampling: u = clip(v + eps, +-[steer_max, accel_max]), eps ~ N(0, diag(sigma_eps^2)).
 * Chance constraint and DCBF: per-wall violation probability delta gives the back-off
 *   nu = sqrt(2) erfinv(1 - 2 delta) (backoff = 0) or sqrt((1-delta)/delta) (backoff = 1,
 *   Remark 1); h = max(w_T - nu sigma_y, 0)^2 - e_y^2 (eq. 33) on the mean lateral deviation e_y and
 *   its std sigma_y; C_safe = C_cbf max(-h_t + (1 - gamma) h_{t-1}, 0) (eqs. 24-25).
 * Costs: q = q_vx (vx - v_goal)^2 + q_vy vy^2 + q_r r^2 + q_ey e_y^2 + q_epsi 2 (1 - cos e_psi)
 *   + C_obs [|e_y| >= w_T] on the mean state (eqs. 27-28); phi = phi_scale q; control cost
 *   gamma_u v^T Sigma_eps^-1 u (eq. 8).
 * Shield repair: shield_iters damped Gauss-Newton steps
 *   u <- clip(u - max(r, 0) g / (|g|^2 + shield_gmin^2)) on the one-step DCBF residual
 *   r(u) = -h(f(xbar_t, u); sigma_t) + (1 - gamma) h_t of each sampled control, g = dr/du by
 *   central differences of step shield_fd; 0 iterations disables it.
 * Launch shape: lanes = lanes per sample (8, 16, 32 or 64), 0 = choose automatically.
 * Belief propagation (Alg. 2): belief = 0 carries M persistent particles through the steps;
 *   belief = 1 redraws them at every step t >= 1 from N(xbar_t, Sigma_t), the mean and full 6x6
 *   sample covariance of the current set (standard normals from Philox tags 4 and 5), before
 *   propagating them; belief = 2 (requires M = 12) replaces the particles by the 12 sigma points
 *   mean +- sqrt(6) L e_i of the belief (equal weights 1/12), propagated without noise, with the
 *   disturbance covariance added to the propagated covariance.
 * Obstacles: n_obs (0..4) circular obstacles, obs[3i..3i+2] = centre x, y and radius, each a
 *   further chance constraint (eq. 16: h = min over the constraints): with d the distance of the
 *   mean position to the centre and sigma the spread along the direction from the centre,
 *   h_i = max(d - nu sigma, 0)^2 - r^2 (the quadratic form of eq. 33), and the collision indicator
 *   adds C_obs while the mean is inside.
 * Disturbance variants: crn = 1 gives every sample the same disturbance draws (common random
 *   numbers: the counter's sample word is 0); sigma_w_speed = kappa makes the disturbance depend
 *   on the state, p(w | x) with std sigma_w (1 + kappa |vx|) at the step's starting state.
 * Repair of the updated sequence (the local repair of v+ from the state estimate in Alg. 1):
 *   local_repair = 1 or 2 runs, after the update, one more rollout from (xbar_0, Sigma_0) whose
 *   control at step t is clip(v+_t) repaired as above (shield_iters >= 1 required) against the
 *   belief of that rollout, and replaces v+ by the repaired sequence v_safe (held in single
 *   precision before it is widened back; v_safe_0 is the returned command and the next warm
 *   start is v_safe).  The rollout's M particles draw their disturbance from their own stream:
 *   the Philox key of seed ^ 0x5DEECE66DA3B9F1B, sample word 0.  local_repair = 1 keeps the
 *   repair of every sampled control as well; 2 samples without it (repair of the update only).
 *   Not available in batches (bss_batch_create rejects such contexts).
 * Half-space constraints on the whole state (the general back-off constraint of eq. 11 with the
 *   heuristic of eq. 13 on the belief z = [xbar; vec Sigma] of eq. 12): n_con (0..4) constraints
 *   c_i(x) = a_i^T x - b_i <= 0, a_i = con_a[6i..6i+5] over (X, Y, psi, vx, vy, r), b_i =
 *   con_b[i].  Each is a further term of h = min_i h_i (eq. 16) with
 *   h_i = b_i - a_i^T xbar - nu sqrt(a_i^T Sigma a_i), Sigma the full 6x6 covariance of the belief,
 *   in the units of c_i (scale a_i and b_i to weigh it against the track's squared-metre form).
 *   The belief keeps a_i^T Sigma a_i per record (the variance of the particles' projections
 *   a_i^T x^n, the same unbiased estimate as the covariance; with sigma points plus a_i^T Q a_i of
 *   the disturbance).  Such instances run in rollout variants with the constraints compiled in
 *   (batches and the server run them for all their members when one is constrained); the staged
 *   bss_dev_score and bss_dev_repair reject n_con > 0. * Vehicle (the Simulation Study's model): vehicle = 0 is the 6-state car above; vehicle = 1 is
 *   the paper's 8-state single-track vehicle with wheel speeds in the road-aligned frame,
 *   x = [vX, vY, r, wF, wR, epsi, eY, s] (body velocities, yaw rate, front and rear wheel speeds,
 *   heading error and lateral deviation from the centerline, path coordinate), u = [steer,
 *   throttle in +-accel_max]: wheel-frame slips (Rw w - v_x) / max(v_x, v_min) and slip angles
 *   -atan(v_y / max(v_x, v_min)), magic-formula pure-slip forces mu Fz D sin(C atan(Bz -
 *   E(Bz - atan Bz))) (pac_B..pac_E, static axle loads), combined by the friction ellipse
 *   Fy = Fy0 sqrt(1 - (Fx0 / (mu D Fz))^2); m vX' = m r vY + Fxf cos d - Fyf sin d + Fxr,
 *   m vY' = -m r vX + Fxf sin d + Fyf cos d + Fyr, Iz r' = lf (Fxf sin d + Fyf cos d) - lr Fyr,
 *   Iw wF' = -Rw Fxf, Iw wR' = throttle T_max - Rw Fxr; s' = (vX cos epsi - vY sin epsi) /
 *   (1 - kappa eY), eY' = vX sin epsi + vY cos epsi, epsi' = r - kappa s' with the centerline
 *   curvature kappa(s) = (2 pi / track_len)(1 + kappa_amp sin(4 pi s / track_len)); n_sub
 *   explicit-midpoint substeps per period dt; the disturbance acts on (vX, vY, r).  The belief is
 *   the mean of the 8 states and the variance of eY (sigma_y), the barrier eq. 33 and the
 *   running cost (x - x_g)^T Q (x - x_g) + C_obs [|eY| >= w_T] with x_g = (v_goal, 0, ...) and
 *   Q = diag(q_vx, q_vy, q_r, 0, 0, q_epsi, q_ey, 0) (eq. 27).  The state estimate has 8 entries
 *   and is known exactly (Sigma0 must be NULL); the shield repair, obstacles, half-space
 *   constraints, belief != 0, sigma_w_speed, the repair of the update, batches and the server
 *   are not available for it (BSS_E_INVAL).
 */
typedef struct bss_params {
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
    int32_t lanes;
    int32_t belief;
    int32_t crn;
    double sigma_w_speed;
    int32_t n_obs;
    double obs[12];
    int32_t local_repair;
    int32_t n_con;
    double con_a[24];
    double con_b[4];
    int32_t vehicle;
    double Rw, Iw, T_max;
    double pac_B, pac_C, pac_D, pac_E;
    double track_len, kappa_amp;
    int32_t n_sub;
} bss_params;

/* Optional device-memory provider (e.g. a framework's caching allocator).  alloc returns a
 * device pointer of at least `bytes` bytes (256-byte aligned) or NULL; release frees it. */
typedef struct bss_allocator {
    void* (*alloc)(size_t bytes, void* user);
    void (*release)(void* ptr, void* user);
    void* user;
} bss_allocator;

/* Device buffers owned by a context (valid until bss_destroy).  Layouts are row-major:
 *   v      [T][2]       double  mean control sequence (warm start).  Each solve writes the
 *                               updated sequence into the other buffer of a ping-pong pair, so
 *                               this pointer changes after every solve: query it again.
 *   u      [K][T][2]    float   sampled (clipped, repaired) controls of the last solve (written
 *                               only when BSS_OUT_CONTROLS is set)
 *   mom    [K][T+1][9]  double  belief per sample and step: mean X, Y, psi, vx, vy, r, then
 *                               Sigma_XX, Sigma_XY, Sigma_YY; record 0 is the given estimate
 *                               (written when BSS_OUT_BELIEFS is set or the records do not fit
 *                               on chip)
 *   S      [K]          double  trajectory costs of the last solve
 *   stats  [8]          double  S_min, Z = sum_k w_k, ESS = Z^2/sum w^2, #finite costs,
 *                               status (0 ok, 5 numeric), v+_0 (steer, accel), number of
 *                               DCBF violations (as bss_info.dcbf_violations)
 *   x0     [6]          double  staging slot for the state estimate ([8] for vehicle = 1)
 *   Sigma0 [36]         double  staging slot for the state-estimate covariance
 *   con_var [K][T+1][n_con] double  a_i^T Sigma a_i of the half-space constraints per record
 *                               (NULL when n_con = 0); record 0 holds a_i^T Sigma0 a_i     */
typedef struct bss_buffers {
    double* v;
    float* u;
    double* mom;
    double* S;
    double* stats;
    double* x0;
    double* Sigma0;
    int32_t v_shift;   /* warm-start shifts pending on v: the mean sequence is
                          v[min(t + v_shift, T - 1)] */
    double* con_var;   /* [K][T+1][n_con] a_i^T Sigma a_i of the half-space constraints per
                          sample and record, or NULL when n_con = 0 */
} bss_buffers;

/* Optional per-solve outputs in device memory (bss_set_outputs); the update does not need them. */
#define BSS_OUT_CONTROLS 1   /* sampled controls u [K][T][2] */
#define BSS_OUT_BELIEFS 2    /* belief records mom [K][T+1][9] and con_var [K][T+1][n_con]; without
                                it a single context's solve keeps them in on-chip memory when they
                                fit beside the resident blocks (then mom and con_var are not
                                written), and in its device buffers otherwise */

/* Result summary of a solve (host): S_min = min_k S_k and Z = sum_k exp(-(S_k - S_min)/lambda)
 * (eq. 7), ess = Z^2 / sum_k w_k^2, n_finite = samples with a finite cost;
 * dcbf_violations = the solve's (sample, step) transitions whose belief violated the linear
 * class-kappa condition h_{t+1} >= (1 - gamma) h_t (eq. 24, the ones C_safe penalises);
 * kernel_ms = the rollout kernel's time of the last solve (HIP events) while timing is enabled
 * (bss_timing_enable), else -1; records_on_chip = 1 when the context's solves keep the belief
 * records in on-chip memory (BSS_OUT_BELIEFS off and room for them). */
typedef struct bss_info {
    double S_min, Z, ess;
    int32_t n_finite;
    int32_t lanes, ppl;       /* launch shape used: lanes per sample, particles per lane */
    int32_t split;            /* 1 when the disturbance normals came from separate waves */
    int32_t dcbf_violations;
    float kernel_ms;
    int32_t records_on_chip;
} bss_info;

typedef struct bss_ctx bss_ctx;

/* Fill *p with the reference problem: the car and track of the small single-solve workload
 * (K=256, M=16, T=30; 30 m x 20 m ellipse, w_T = 2 m; delta = 0.05; gamma = 0.2; lambda = 1). */
void bss_params_default(bss_params* p);

/* Check a parameter set without touching the GPU.  BSS_E_INVAL with a message if any field is
 * out of range (sizes >= 1, K <= 2^20, T <= 256, M <= 512, 0 < delta < 0.5, 0 < gamma <= 1, lambda > 0,
 * dt > 0, finite non-negative noise std, and a track whose ellipse keeps a unique nearest point
 * inside the band: min(a,b)^2 / max(a,b) > half_width). */
bss_status bss_validate(const bss_params* p);

/* Back-off coefficient nu for the parameter set (host computation, Remark 1). */
bss_status bss_backoff(const bss_params* p, double* nu_out);

/* Create a context on the current HIP device (the device is chosen by the caller with hipSetDevice
 * before the call; the context stays on it).  `alloc` may be NULL (hipMalloc is used); `stream`
 * is a hipStream_t (NULL = the null stream) on which every later call of this context enqueues
 * its work.  The mean control sequence starts at zero (Alg. 1's initial v) and the solve index
 * at 0.
 * Errors: BSS_E_INVAL (parameters, out == NULL), BSS_E_NOMEM, BSS_E_DEVICE. */
bss_status bss_create(const bss_params* p, const bss_allocator* alloc, void* stream,
                      bss_ctx** out);

/* Change the stream of a context (subsequent calls enqueue there). */
bss_status bss_set_stream(bss_ctx* c, void* stream);

/* One solve from host inputs, synchronous: x0[6] the state estimate (x0[8] for vehicle = 1),
 * Sigma0 a 6x6 row-major covariance or NULL (known state), u0_out[2] receives the command v+_0,
 * info may be NULL.
 * Updates the mean control sequence in place (Alg. 1: v <- v_safe) and advances the solve index.
 * Errors: BSS_E_INVAL (non-finite x0 or Sigma0, NULL pointers), BSS_E_NUMERIC (every cost was
 * non-finite; v unchanged), BSS_E_DEVICE. */
bss_status bss_solve(bss_ctx* c, const double x0[6], const double* Sigma0, double u0_out[2],
                     bss_info* info);

/* One solve from device-resident inputs, asynchronous on the context's stream: x0_dev [6] ([8]
 * for vehicle = 1) and Sigma0_dev [36] (or NULL) are device pointers that must stay valid until
 * the work completes.  Results land in the context's buffers (bss_get_buffers); the status word
 * stats[4] is 5 when every cost was non-finite (then v is unchanged).  Errors: BSS_E_INVAL,
 * BSS_E_DEVICE. */
bss_status bss_solve_async(bss_ctx* c, const double* x0_dev, const double* Sigma0_dev);

/* Receding-horizon warm start (Alg. 1: the updated sequence seeds the next control period; after
 * its first control has been applied the sequence moves one step): v_t <- v_{t+1} for t < T-1;
 * v_{T-1} keeps its value.  The shift is recorded in the context and applied when the next solve
 * reads v (no kernel is launched); bss_get_controls returns the shifted sequence. */
bss_status bss_step_shift(bss_ctx* c);

/* Select the optional per-solve outputs (BSS_OUT_CONTROLS | BSS_OUT_BELIEFS, both on after
 * bss_create).  The solve's costs, update, command and stats are the same bit for bit either way.
 * Errors: BSS_E_INVAL (unknown flags), BSS_E_STATE (context in a batch), BSS_E_DEVICE. */
bss_status bss_set_outputs(bss_ctx* c, int32_t flags);

/* Device buffers of the context (see bss_buffers). */
bss_status bss_get_buffers(const bss_ctx* c, bss_buffers* out);

/* Copy the mean control sequence [T][2] to / from host memory (synchronous). */
bss_status bss_get_controls(bss_ctx* c, double* v_host);
bss_status bss_set_controls(bss_ctx* c, const double* v_host);

/* Solve index used for the random-number counters of the next solve (resuming a context at a
 * given index reproduces its noise exactly). */
bss_status bss_set_solve_index(bss_ctx* c, uint32_t s);
bss_status bss_get_solve_index(const bss_ctx* c, uint32_t* s);

/* Synchronise the stream and read the stats of the last solve into *info. */
bss_status bss_get_info(bss_ctx* c, bss_info* info);

/* Kernel timing: when enabled, HIP events bracket the rollout kernel of every solve on the
 * context's stream.  bss_timing_read synchronises, returns the summed rollout-kernel time in ms
 * and the number of solves measured since the last read, and resets the accumulators. */
bss_status bss_timing_enable(bss_ctx* c, int32_t enable);
bss_status bss_timing_read(bss_ctx* c, double* rollout_ms_total, int32_t* count);

/* Force the launch shape (lanes per sample 8/16/32/64; 0 restores the automatic choice). */
bss_status bss_set_lanes(bss_ctx* c, int32_t lanes);

/* Force lanes per sample (0, 8, 16, 32, 64) and particles per lane (0, 1, 2, 4, 8; 0 = automatic;
 * a nonzero ppl takes precedence over lanes) and the noise split (-1 automatic, 0 off, 1 on): with
 * the split, each block of 512 threads has a second set of waves that generates the disturbance
 * normals one step ahead, which doubles the waves per SIMD of a launch too small to fill the chip
 * (automatic: when the launch has fewer than two waves per SIMD; never for the shielded loop
 * nor for constraints together with re-sampling; with re-sampling the noise waves also draw the
 * re-sampling normals).
 * The M particles of a sample are spread over L lanes with P = ceil(M / L) per lane.  Results
 * depend on the shape only through the summation order of the per-step moments (not on the
 * split).  Errors: BSS_E_INVAL (values, or M > 64 P), BSS_E_STATE (context in a batch). */
bss_status bss_set_shape(bss_ctx* c, int32_t lanes, int32_t ppl, int32_t split);

/* Destroy a context and free its buffers (resource management; no passage of the paper).  NULL is
 * accepted; a context that belongs to a batch is left alone: destroy the batch first.  Work
 * enqueued on the context's stream is waited for before its buffers are released. */
void bss_destroy(bss_ctx* c);

/* ---- batches: many controllers, one solve launch and one merge launch ---------------------------
 *
 * A batch runs one solve of each of n contexts (each with its own K, M, T, costs, seed and warm
 * start, Alg. 1 per context) in two kernel launches: the rollout/scoring grid is the union of the
 * contexts' blocks (ordered by their work, longest first) and the merge grid the union of their
 * control entries.  All per-solve state (mean-sequence buffer, pending shift, solve index) advances on the
 * device, so the two launches can be captured once in a HIP graph and replayed.  Each context of a
 * batch computes exactly what it computes alone with the same launch shape.  While a context
 * belongs to a batch, its own solve and state calls return BSS_E_STATE. */
typedef struct bss_batch bss_batch;

/* Group n contexts (distinct, not in another batch, all on the current device) into a batch whose
 * work is enqueued on the stream of ctxs[0].  ppl: particles per lane used by every member (1, 2,
 * 4 or 8; 0 = automatic; bss_batch_tune measures the candidates, bss_batch_set_member_ppl sets
 * one per member).  shift_after = 1 leaves one
 * warm-start shift pending after each solve (the receding-horizon loop of a controller), 0 none.
 * The batch takes over each context's mean sequence, shift and solve index, and hands them back
 * in bss_batch_destroy.  Errors: BSS_E_INVAL, BSS_E_STATE, BSS_E_NOMEM, BSS_E_DEVICE. */
bss_status bss_batch_create(bss_ctx* const* ctxs, int32_t n, int32_t ppl, int32_t shift_after,
                            bss_batch** out);

/* Device array x0[n][6] (double) read by each batched solve: member i's state estimate is row i.
 * The caller may write it with its own kernels or copies, ordered before bss_batch_solve on the
 * batch's stream.  The batched solve uses a known state (Sigma0 = 0). */
bss_status bss_batch_states(bss_batch* b, double** x0_dev);

/* Copy x0_host[n][6] into the state array (synchronous).  Errors: BSS_E_INVAL (non-finite). */
bss_status bss_batch_set_states(bss_batch* b, const double* x0_host);

/* Enqueue a device-to-device copy of x0_dev[n][6] (double, device memory that stays valid until
 * the copy completes) into the state array on the batch's stream. */
bss_status bss_batch_copy_states(bss_batch* b, const double* x0_dev);

/* Enqueue one solve of every member (asynchronous; replays the captured graph if there is one).
 * Results land in each member's buffers; bss_get_buffers, bss_get_controls and bss_get_info
 * work on members (they synchronise the batch's stream). */
bss_status bss_batch_solve(bss_batch* b);

/* Capture the batch's two launches into a HIP graph used by later bss_batch_solve calls.  The
 * batch's stream must be a created stream (BSS_E_STATE on the null stream). */
bss_status bss_batch_capture(bss_batch* b);

/* Autotuner of the batch's launch.  First one particles-per-lane count P for every member: each
 * candidate with and without the noise split, each as a one-shot grid (one block per table entry)
 * and as a persistent grid (as many blocks as are resident on the device, taking the block
 * table's entries -- most work first -- from a work-queue counter).  Then, for batches whose
 * members neither repair their samples, redraw their particles nor have half-space constraints,
 * each member's own P in the same launch: members grouped by M, the groups in order of their
 * work try every other P on top of the best common one, and a change is kept when the batch gets
 * faster by more than 1 %.  Every candidate is timed on the batch itself (trial solves whose
 * state changes, mean sequences and stats are undone; the members' cost and belief buffers hold
 * a trial solve until the next one), and the fastest layout is kept.  The choice is cached for
 * the process per batch signature (device, and each member's K, M, T and variant flags in order):
 * a later batch of the same signature takes it without trial solves.  *ppl_out (may be NULL)
 * receives the common P, or 0 when the members run their own (bss_batch_member_shape).  Call
 * before bss_batch_capture. */
bss_status bss_batch_tune(bss_batch* b, int32_t* ppl_out);

/* Solve grid of the batch's rollout launch (the propagation of Alg. 2 for every member): 0 =
 * one block per entry of the block table, 1 = persistent (as many blocks as are resident on the
 * device, each taking the next entry, most work first, from a work-queue counter that a kernel
 * launched first resets).  Results are the same bit for bit.  The persistent grid is built for
 * batches whose members neither repair their samples, redraw their particles nor have
 * half-space constraints (BSS_E_INVAL otherwise).  Call before bss_batch_capture (BSS_E_STATE
 * after).  bss_batch_tune chooses it by measurement. */
bss_status bss_batch_set_grid(bss_batch* b, int32_t persistent);

/* Each member's own particles per lane, run in one launch: ppl[n], each 1, 2, 4 or 8 with
 * ceil(M_i / ppl[i]) <= 64 (BSS_E_INVAL otherwise); the members' lanes per sample follow (the
 * smallest power of two >= 8 holding M_i).  A member computes exactly what it computes alone with
 * the same lanes and particles per lane.  For batches whose members neither repair their
 * samples, redraw their particles nor have half-space constraints (BSS_E_INVAL otherwise).  Call
 * before bss_batch_capture (BSS_E_STATE after). */
bss_status bss_batch_set_member_ppl(bss_batch* b, const int32_t* ppl);

/* Lanes per sample and particles per lane of member i (0 <= i < n) in the current layout (either
 * may be NULL). */
bss_status bss_batch_member_shape(const bss_batch* b, int32_t i, int32_t* lanes, int32_t* ppl);

/* Number of solve blocks, particles per lane (0 when the members run their own) and grid flags of
 * the batch's current layout (any may be NULL): *split bit 0 = noise split, bit 1 = persistent
 * grid. */
bss_status bss_batch_info(bss_batch* b, int32_t* nblocks, int32_t* ppl, int32_t* split);

/* Synchronise the batch's stream, hand each member its state back and free the batch (NULL is
 * accepted). */
void bss_batch_destroy(bss_batch* b);

/* ---- serving: many vehicles, solves batched as their requests arrive ------------------------
 *
 * Each vehicle runs the receding-horizon loop of Alg. 1 on its own problem (track, car, noise,
 * seed: a bss_params); every request asks for one solve of that vehicle from a state estimate, with
 * its own sample count K, particle count M and risk level delta.  The vehicle's mean control
 * sequence stays in device memory between requests and is warm-started (shifted by one step)
 * after every solve; its solve index advances by one per solve, so a vehicle's results depend only
 * on its own request sequence, never on which other requests shared a launch.
 *
 * Device memory: the resident mean sequences (2 x T x 2 doubles per vehicle) plus hbm_budget bytes
 * of scratch split evenly over n_streams slots.  A request is admitted into a batch while its
 * scratch (belief records, costs and block partials: about 3.7 KB x K at T = 50) fits in the slot.
 * Whenever a slot is free, bss_server_pump launches every admissible pending request (oldest first,
 * at most one per vehicle, at most max_batch) as one solve launch and one merge launch on the slot's
 * stream; slots run concurrently.  Not thread-safe: one thread drives a server. */
typedef struct bss_server bss_server;

typedef struct bss_server_config {
    int32_t n_vehicles;
    int32_t T;            /* horizon shared by every vehicle */
    int32_t K_max, M_max; /* per-request limits */
    int32_t ppl;          /* particles per lane of the batched launches (0 = 4) */
    int32_t n_streams;    /* batches in flight at once, 1..16 */
    int32_t max_batch;    /* requests per launch, 1..4096 */
    uint64_t hbm_budget;  /* bytes of device scratch for in-flight solves */
} bss_server_config;

/* A finished request: its command v+_0, BSS_OK or BSS_E_NUMERIC (no finite cost; the warm start
 * was kept), and the host steady-clock time (seconds) at which the server saw it complete. */
typedef struct bss_completion {
    int64_t req;
    int32_t vehicle;
    int32_t status;
    double u0[2];
    double t_done;
} bss_completion;

/* 256 vehicles, T = 50, K <= 8192, M <= 128, 4 particles per lane, 2 streams, batches of up to
 * 256, 32 GiB of scratch. */
void bss_server_config_default(bss_server_config* c);

/* Create a server on the current device.  vehicles[n_vehicles] are copied; their K, M and T fields
 * are ignored (validated as K_max, M_max, T), delta is replaced per request.  Mean sequences start
 * at zero, solve indices at 0.  Errors: BSS_E_INVAL (a budget below one K_max request per stream,
 * M_max above 64 x ppl, invalid vehicle parameters), BSS_E_NOMEM, BSS_E_DEVICE. */
bss_status bss_server_create(const bss_server_config* cfg, const bss_params* vehicles,
                             bss_server** out);

/* Queue one solve of `vehicle` from the state estimate x0[6] (copied).  *req_id (may be NULL)
 * receives the request's id (consecutive from 0).  Nothing is launched until bss_server_pump. */
bss_status bss_server_submit(bss_server* s, int32_t vehicle, int32_t K, int32_t M, double delta,
                             const double x0[6], int64_t* req_id);

/* Retire completed batches (their requests become pollable) and launch new batches on free slots.
 * Never blocks.  *n_launched (may be NULL) receives the number of requests launched. */
bss_status bss_server_pump(bss_server* s, int32_t* n_launched);

/* Move up to max completions into out[]; returns how many. */
int32_t bss_server_poll(bss_server* s, bss_completion* out, int32_t max);

/* Pump until nothing is pending or in flight (completions stay pollable). */
bss_status bss_server_drain(bss_server* s);

/* Mean control sequence [T][2] of an idle vehicle (no request pending or in flight; BSS_E_STATE
 * otherwise), with its pending warm-start shift applied; and setting it (clears the shift). */
bss_status bss_server_get_controls(bss_server* s, int32_t vehicle, double* v_host);
bss_status bss_server_set_controls(bss_server* s, int32_t vehicle, const double* v_host);

/* Solve index of the vehicle's next solve and its number of unfinished requests. */
bss_status bss_server_vehicle_state(const bss_server* s, int32_t vehicle, uint32_t* solve_index,
                                    int64_t* pending);

/* Replay a request trace in real time: request i is submitted once t_arrival[i] seconds have
 * passed since the call started (non-decreasing times), the server is pumped continuously, and
 * latency_s[i] = completion time - scheduled arrival.  x0 is [n][6]; u0_out [n][2] and status_out
 * [n] may be NULL.  Drains the server first; returns when every request has completed. */
bss_status bss_server_replay(bss_server* s, int64_t n, const double* t_arrival,
                             const int32_t* vehicle, const int32_t* K, const int32_t* M,
                             const double* delta, const double* x0, double* latency_s,
                             double* u0_out, int32_t* status_out);

/* Wait for the work in flight and free the server (NULL is accepted). */
void bss_server_destroy(bss_server* s);

/* ---- one solve that allocates nothing --------------------------------------------------- */

/* Bytes of the library's static per-GPU scratch array: 48 MiB, held on each GPU the library runs
 * on until the process ends. */
#define BSS_NOALLOC_SCRATCH_BYTES ((size_t)48 << 20)

/* For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  One solve of parameter set p from the device-resident
 * state estimate x0_dev [6] ([8] for vehicle = 1; Sigma0_dev [36] or NULL) and mean sequence
 * v_in_dev [T][2] at solve index solve_index: the same kernels and launch shape as bss_solve_async on a context of
 * p whose mean sequence is v_in, with no pending shift, at that solve index, so v_out_dev [T][2]
 * receives that context's v+ and stats_dev [8] its stats (layout of bss_buffers) bit for bit.
 * All pointers are device pointers owned by the caller; v_in_dev and v_out_dev must differ; v_in
 * is only read.  Asynchronous on `stream`: three kernels, no copy, no allocation, no host
 * synchronisation.  Every scratch buffer of the solve (descriptor, grids, belief records,
 * constraint variances, costs, block partials) lives in the library's static array of
 * BSS_NOALLOC_SCRATCH_BYTES on the current GPU (bss_noalloc_scratch_bytes gives a problem's
 * need); calls that overlap on one GPU share it and race, so enqueue them on one stream or
 * order them.  Errors: BSS_E_INVAL for invalid parameters, NULL pointers, v_in_dev == v_out_dev,
 * local_repair != 0, or a problem whose scratch exceeds the array (the message gives both
 * sizes; checked before any device call); BSS_E_DEVICE for a failed launch. */
bss_status bss_solve_noalloc(const bss_params* p, uint32_t solve_index, const double* x0_dev,
                             const double* Sigma0_dev, const double* v_in_dev, double* v_out_dev,
                             double* stats_dev, void* stream);
/* Scratch bytes bss_solve_noalloc needs for p (0 for invalid parameters). */
size_t bss_noalloc_scratch_bytes(const bss_params* p);

/* Message of the last failing call on this thread ("" if none). */
const char* bss_last_error(void);

/* ---- stand-alone device kernels of the solve, for staged checks (all device pointers, work
 *      enqueued on `stream`, n >= 0 elements) ------------------------------------------------ */

/* Philox4x32-10 (Salmon et al., SC'11) of n counters ctr[n][4] under key (lo32 seed, hi32 seed)
 * into out[n][4]. */
bss_status bss_dev_philox(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n,
                          void* stream);
/* Four Box-Muller normals per counter: z[n][4] (single precision) from the block's words
 * (r0, r1) and (r2, r3) with uniforms ((r >> 9) + 1/2) 2^-23. */
bss_status bss_dev_normals(uint64_t seed, const uint32_t* ctr, float* z, int64_t n, void* stream);
/* The disturbance normals of a solve (the "sample w" line of the propagation algorithm, Alg. 2,
 * under the counter contract of bss_dev_philox: word 0 = t, word 1 = 3q + b, word 2 = k, or 0
 * with crn != 0, word 3 = (1 << 28) | (solve_index & 0x0FFFFFFF)), computed by the solve
 * kernel's own code path for a launch of `lanes` lanes per sample and `ppl` particles per lane
 * (lanes in {8, 16, 32, 64}, ppl in {1, 2, 4, 8}, lanes * ppl >= M; BSS_E_INVAL otherwise).
 * Particle quad q = m / 4 draws the three blocks b = 0, 1, 2 and particle 4q + i takes normals
 * 3i .. 3i + 2 of their twelve (block b: normals 4b .. 4b + 3 as bss_dev_normals).
 * Outputs (device, caller-owned): words[K][T][3 ceil(M / 4)][4] (the raw Philox words of every
 * block), w[K][T][M][3] (single precision, before the scaling by sigma_w). */
bss_status bss_dev_disturbance(uint64_t seed, uint32_t solve_index, int32_t K, int32_t M,
                               int32_t T, int32_t crn, int32_t lanes, int32_t ppl, float* w,
                               uint32_t* words, void* stream);
/* One noise-free single-precision RK2 step of the car: x[n][6], u[n][2] -> xn[n][6]. */
bss_status bss_dev_model_step(const bss_params* p, const float* x, const float* u, float* xn,
                              int64_t n, void* stream);
/* One noise-free single-precision control period of the 8-state vehicle (vehicle = 1; its n_sub
 * midpoint substeps, the Simulation Study's single-track model with wheel speeds): x[n][8]
 * (absolute path coordinate), u[n][2] -> xn[n][8].  BSS_E_INVAL for vehicle != 1. */
bss_status bss_dev_model_step8(const bss_params* p, const float* x, const float* u, float* xn,
                               int64_t n, void* stream);
/* Signed distance to the centerline ellipse and its outward normal, double precision:
 * pts[n][2] -> out[n][3] = (e_y, n_x, n_y). */
bss_status bss_dev_sdf(double a, double b, const double* pts, double* out, int64_t n,
                       void* stream);
/* Trajectory costs from given beliefs and controls (the scoring stage alone):
 * mom[K][T+1][9], u[K][T][2] (float), v[T][2] -> S[K]. */
bss_status bss_dev_score(const bss_params* p, const double* mom, const float* u, const double* v,
                         double* S, void* stream);
/* MPPI update from given costs and controls: S[K], u[K][T][2] (float); v[T][2] updated in place,
 * stats[8] as in bss_buffers.  workspace: at least bss_dev_update_workspace(K, T) bytes of
 * device memory (scratch, caller-owned). */
size_t bss_dev_update_workspace(int32_t K, int32_t T);
bss_status bss_dev_update(const bss_params* p, const double* S, const float* u, double* v,
                          double* stats, void* workspace, void* stream);
/* Shield repair of n controls from given beliefs: mom[n][9], u_in[n][2] -> u_out[n][2]
 * (double precision). */
bss_status bss_dev_repair(const bss_params* p, const double* mom, const double* u_in,
                          double* u_out, int64_t n, void* stream);

#ifdef __cplusplus
}
#endif
#endif
