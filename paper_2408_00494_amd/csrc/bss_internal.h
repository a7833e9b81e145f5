// bss_internal.h -- structures shared between the C ABI layer and the HIP kernels of libbssmppi.
//
// The rollout works in single precision on per-particle state; every per-(sample, step) scalar
// (moments, scores, the shield repair) and the K-reduction work in double precision.
//
// Every solve launch is descriptor-driven: an InstanceDesc in device memory describes one problem
// (a context), a BlockDesc maps each block of the solve grid to (instance, first sample), and a
// MergeDesc maps each wave of the merge grid to (instance, control entry).  A single context is
// a batch of one; a batch of uneven instances runs in the same two launches.  The per-solve state
// (which ping-pong buffer holds the mean sequence, pending warm-start shifts, the solve index)
// lives in the descriptor and is advanced on the device, so a batched launch can be captured in a
// graph and replayed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace bss {

constexpr int kMaxObstacles = 4;
constexpr int kMaxCon = 4;         // half-space constraints a_i^T x <= b_i on the whole state

// Constants of the single-track car in the form the single-precision particle integrator uses:
// forces are divided by the mass, so the saturations and stiffnesses are accelerations.
struct CarF32 {
    float dt, half_dt;
    float lf, lr;
    float cf_m, cr_m;          // Cf / m, Cr / m
    float fF_max, fR_max;      // mu g lr / L, mu g lf / L
    float m_Iz;                // m / Iz
    float v_min;
};

// Constants of the 8-state single-track vehicle with wheel speeds (vehicle = 1) in the form the
// single-precision integrator uses (built on the host).
struct Car8F32 {
    float h, half_h;           // substep dt / n_sub and half of it
    int32_t n_sub;             // midpoint substeps per control period
    float lf, lr, inv_m, inv_Iz;
    float Rw, Rw_Iw, Tmax_Iw;  // wheel radius, Rw / Iw, T_max / Iw
    float muFzf, muFzr;        // mu times the static load of each axle
    float inv_fmaxf, inv_fmaxr;  // 1 / (mu D Fz) per axle (friction-ellipse semi-axis)
    float B, C, D, E;          // magic-formula coefficients
    float v_min;               // floor of the slip denominators
    float kappa0, kappa_amp;   // curvature (2 pi / L)(1 + a sin(...))
    float s_rev;               // 2 / L: revolutions of sin(4 pi s / L) per metre
};

// The centerline ellipse in the form the signed distance uses (built on the host): semi-axes
// ordered e0 >= e1 for the nearest-point solve, and the reciprocals it multiplies by.
struct EllipseF64 {
    double inv_a2, inv_b2;                      // 1/a^2, 1/b^2 (a along X, b along Y)
    double e0, e1;                              // larger and smaller semi-axis
    double inv_e0, inv_e1, inv_e0sq, inv_e1sq;  // 1/e0, 1/e1, 1/e0^2, 1/e1^2
    double r0;                                  // (e0/e1)^2
    double inv_denom0;                          // 1/(e0^2 - e1^2) (0 for a circle)
    int32_t swap;                               // 1 when b > a: the solve runs on (Y, X)
};

inline EllipseF64 make_ellipse(double a, double b)
{
    EllipseF64 E;
    E.inv_a2 = 1.0 / (a * a);
    E.inv_b2 = 1.0 / (b * b);
    E.swap = b > a ? 1 : 0;
    E.e0 = E.swap ? b : a;
    E.e1 = E.swap ? a : b;
    E.inv_e0 = 1.0 / E.e0;
    E.inv_e1 = 1.0 / E.e1;
    E.inv_e0sq = 1.0 / (E.e0 * E.e0);
    E.inv_e1sq = 1.0 / (E.e1 * E.e1);
    E.r0 = (E.e0 / E.e1) * (E.e0 / E.e1);
    const double den = E.e0 * E.e0 - E.e1 * E.e1;
    E.inv_denom0 = den > 0.0 ? 1.0 / den : 0.0;
    return E;
}

// Everything the double-precision per-(sample, step) code needs: model (for the shield's mean
// prediction), costs, barrier and repair settings.
struct ScoreF64 {
    double m, Iz, lf, lr, Cf, Cr, mu, g, v_min, dt;
    double steer_max, accel_max;
    double inv_var0, inv_var1;      // 1 / sigma_eps^2 (0 where the std is 0)
    double gamma_u, v_goal, q_vx, q_vy, q_r, q_ey, q_epsi, C_cbf, C_obs, phi_scale;
    double ell_a, ell_b, half_width;
    EllipseF64 ell;                 // the same ellipse, prepared for the signed distance
    double nu, gamma, lambda;
    int32_t shield_iters;
    double shield_gmin, shield_fd;
    int32_t n_obs;                  // circular obstacles: centre (obs[3i], obs[3i+1]), radius obs[3i+2]
    double obs[3 * kMaxObstacles];
    // derived on the host: lateral force limits mu m g lr / (lf + lr), mu m g lf / (lf + lr), and
    // 1 / m, 1 / Iz (the double-precision model multiplies instead of dividing)
    double Ffm, Frm, inv_m, inv_Iz;
    // half-space constraints: a_i = con_a[6i..6i+5] over (X, Y, psi, vx, vy, r), bound con_b[i]
    int32_t n_con;
    double con_a[6 * kMaxCon];
    double con_b[kMaxCon];
};

// One problem instance (device memory).
struct InstanceDesc {
    // sizes and launch shape: lanes per sample and P, particles per lane (the kernel's template
    // parameter, except in the per-instance variant, which dispatches on this field)
    int32_t K, M, T, lanes, ppl;
    int32_t nblocks;               // solve blocks of this instance (= number of partials)
    int32_t x0_index;              // state estimate at x0_base + 6 x0_index (launch argument)
    int32_t rec_lds;               // 1: belief records (and constraint variances) kept in the
                                   // block's LDS after the controls (or the noise ring) instead
                                   // of mom / cvar; the launch's LDS includes them
    // per-solve state, advanced on the device by the last merge block of the instance
    int32_t cur;                   // v[cur] holds the mean sequence
    int32_t vshift;                // pending warm-start shifts: read v[min(t + vshift, T - 1)]
    uint32_t solve_index;          // Philox word 3 (low 28 bits)
    uint32_t done;                 // merge blocks finished in the current launch
    int32_t shift_after;           // 1: leave one warm-start shift pending after the solve
    int32_t status;                // 0 ok, 5 no finite cost (v unchanged)
    int32_t belief;                // 0 persistent particles, 1 Gaussian re-sampling every step
    int32_t crn;                   // 1: disturbance counters use sample word 0 for every sample
    // random numbers and model
    uint32_t key0, key1;           // Philox key = (lo32 seed, hi32 seed)
    float steer_max, accel_max;
    float sig_eps0, sig_eps1;
    float sig_w0, sig_w1, sig_w2;
    float sig_w_speed;             // disturbance std factor 1 + sig_w_speed |vx|
    int32_t vehicle;               // 0 the 6-state car, 1 the 8-state vehicle (car8, own kernel)
    CarF32 car;
    Car8F32 car8;
    ScoreF64 sc;
    // buffers
    double* v[2];                  // ping-pong pair of mean sequences [T][2]
    float* u;                      // [K][T][2] copy of the sampled controls, or nullptr
    double* mom;                   // [K][T+1][9] beliefs (written by the loop, read by scoring)
    double* cvar;                  // [K][T+1][n_con] a_i^T Sigma a_i, or nullptr without
                                   // half-space constraints
    double* S;                     // [K] trajectory costs
    double* partial;               // [nblocks][2T + 5] per-block log-sum-exp partials
    double* stats;                 // [8]: S_min, Z, ESS, #finite, status, v+_0 (2),
                                   //      DCBF violations
};

struct BlockDesc {
    int32_t inst;                  // instance index
    int32_t k0;                    // first sample of the block
};

struct MergeDesc {
    int32_t inst;                  // instance index
    int32_t col;                   // control entry 2t + j
};

// Per-block partial of the K-reduction (weights relative to the block's own minimum cost m_b):
//   [0, 2T)  N_i = sum_k w_k (u_{k,i} - v_i),   [2T] Z_b = sum w_k,   [2T+1] sum w_k^2,
//   [2T+2]   number of finite costs,            [2T+3] m_b (+inf if none is finite),
//   [2T+4]   number of the block's (sample, step) transitions whose belief violated the DCBF
//            condition h_{t+1} >= (1 - gamma) h_t.
constexpr int kPartialTail = 5;
__host__ __device__ inline int partial_stride(int T) { return 2 * T + kPartialTail; }

// samples per block of the partial kernel used for stand-alone K-reductions
constexpr int kPartialSlice = 16;

// lanes per sample (L) and particles per lane (P) of one rollout launch; split: 512-thread
// blocks whose second half generates the disturbance normals one step ahead (non-shielded only)
struct LaunchShape {
    int lanes;
    int ppl;
    bool split;
};

constexpr int kMaxT = 256;
// LDS budget of a solve block's controls and noise ring (the shape choice keeps several blocks on a
// CU within it)
constexpr size_t kMaxLds = 65536;

// Moment exchange of the solve kernel: each lane stores its partial moment sums in its group's
// rows (the L lanes' entries, then the group total: an odd stride of L + 1 doubles), and the rows
// are totalled in LDS.  Rows: the nine moment sums, and in the constraint variants the constraints'
// sums of squares of the projections; then the group's reference position (two doubles).
constexpr int moment_rows(bool con) { return con ? 9 + kMaxCon : 9; }
constexpr int moment_region_doubles(int lanes, bool con) { return moment_rows(con) * (lanes + 1) + 2; }

// Dynamic LDS of a solve block (6-state car): costs and weights, the controls, with the noise
// split the ring of normals (three per particle and slot, nine with the re-sampling draw's), then
// the moment exchange (two slots with the split: the noise waves total step t's sums while the
// others integrate step t + 1).  con: a constraint variant is launched.
size_t solve_lds_bytes(int lanes, int T, int ppl, bool split, bool resample = false,
                       bool con = false);
// The part the launch shape is chosen by (within kMaxLds): costs, weights, controls and the ring.
size_t solve_base_lds_bytes(int lanes, int T, int ppl, bool split, bool resample = false);
// Whether a split block of this shape fits the LDS of a workgroup beside the static LDS.
bool split_fits(int lanes, int T, int ppl, bool resample, bool con, size_t static_lds);
// Dynamic LDS of a block of the 8-state vehicle's kernel: costs and weights, and the controls.
size_t solve8_lds_bytes(int lanes, int T);
// LDS of the belief records of one block kept on chip (rec_lds): (256 / lanes) samples x (T + 1)
// records x (9 + n_con) doubles.
size_t record_lds_bytes(int lanes, int T, int n_con);
// LDS one workgroup can allocate on gfx950.
constexpr size_t kMaxLdsPerBlock = 163840;
// Static LDS of the solve kernels: the re-sampling sums (the variants with the re-sampling compiled
// in: group sums of 14 values over 8 lanes, one row of 9 doubles per value and group, 32 groups)
// and at most 2 KB of block-level slots in every variant.
constexpr size_t kResampleStaticLds = (size_t)4 * 8 * 14 * 9 * sizeof(double);
constexpr size_t kStaticLdsSlots = 2048;
// requested_split: -1 automatic (split when the launch has fewer than two waves per SIMD), 0 off,
// 1 on (when the ring fits); shield: the sampled controls are repaired (the automatic shape then
// puts eight particles in a lane)
LaunchShape choose_shape(int K, int M, int T, int requested_lanes, int requested_ppl,
                         int requested_split = -1, bool shield = false);
bool split_pays(int nblocks, int lanes, int T, int ppl);
int solve_blocks(int K, int lanes);

// Solve grid: nblocks blocks described by `blocks`; x0_base holds the state estimates (6 doubles
// per instance at x0_index), Sigma0_base the covariances (36 doubles) or nullptr; extra_shift is
// added to every instance's pending shift for this launch.  Variant flags: shield (some instance
// repairs its samples), split (separate noise waves), resample (some instance redraws its
// particles), con (some instance has half-space constraints: the variant with them compiled in;
// with shield or resample that is the generic one, both of those switched at run time).
// ppl: particles per lane of every instance, or 0 to take each instance's from its descriptor
// (plain and split variants only).
// queue (may be null): a zero-initialised counter in device memory for a persistent grid (as
// many blocks as are resident on the device take the block table's entries in order; the
// counter is reset by a kernel launched first, so the pair can be captured in a graph); plain
// and split variants only.
hipError_t launch_solve(const InstanceDesc* inst, const BlockDesc* blocks, int nblocks, int ppl,
                        bool shield, bool split, bool resample, bool con, size_t lds,
                        const double* x0_base, const double* Sigma0_base, int extra_shift,
                        hipStream_t stream, uint32_t* queue = nullptr);
// the solve launch of one particles-per-lane count (each compiled in its own translation unit)
hipError_t launch_solve_p1(const InstanceDesc* inst, const BlockDesc* blocks, int nblocks,
                           bool shield, bool split, bool resample, bool con, size_t lds,
                           const double* x0_base, const double* Sigma0_base, int extra_shift,
                           uint32_t* queue, hipStream_t stream);
hipError_t launch_solve_p2(const InstanceDesc* inst, const BlockDesc* blocks, int nblocks,
                           bool shield, bool split, bool resample, bool con, size_t lds,
                           const double* x0_base, const double* Sigma0_base, int extra_shift,
                           uint32_t* queue, hipStream_t stream);
hipError_t launch_solve_p4(const InstanceDesc* inst, const BlockDesc* blocks, int nblocks,
                           bool shield, bool split, bool resample, bool con, size_t lds,
                           const double* x0_base, const double* Sigma0_base, int extra_shift,
                           uint32_t* queue, hipStream_t stream);
hipError_t launch_solve_p8(const InstanceDesc* inst, const BlockDesc* blocks, int nblocks,
                           bool shield, bool split, bool resample, bool con, size_t lds,
                           const double* x0_base, const double* Sigma0_base, int extra_shift,
                           uint32_t* queue, hipStream_t stream);
// P taken per instance from InstanceDesc::ppl (plain and split variants only)
hipError_t launch_solve_pm(const InstanceDesc* inst, const BlockDesc* blocks, int nblocks,
                           bool shield, bool split, bool resample, bool con, size_t lds,
                           const double* x0_base, const double* Sigma0_base, int extra_shift,
                           uint32_t* queue, hipStream_t stream);
hipError_t launch_merge(const InstanceDesc* inst, const MergeDesc* cols, int ncols,
                        int extra_shift, hipStream_t stream);
// Repair of the updated sequence of one instance after its merge: `rep` is the instance's repair
// descriptor (one sample, no exploration noise, own key and buffers), `rep_block` its one-block
// grid {0, 0}; lds is the dynamic LDS of an unsplit launch of the instance's shape.
hipError_t launch_local_repair(InstanceDesc* inst, InstanceDesc* rep, const BlockDesc* rep_block,
                               int T, int ppl, bool resample, bool con, size_t lds,
                               const double* x0_base, const double* Sigma0_base,
                               hipStream_t stream);

// stand-alone kernels for staged checks
hipError_t launch_score(int K, int T, const ScoreF64& sc, const double* mom, const float* u,
                        const double* v, double* S, hipStream_t stream);
hipError_t launch_partials(int K, int T, double lambda, const double* S, const float* u,
                           const double* v, double* partial, hipStream_t stream);
hipError_t launch_merge_plain(int T, int G, double lambda, const double* partial,
                              const double* v_in, double* v_out, double* stats,
                              hipStream_t stream);
int partial_blocks(int K);
hipError_t launch_philox(uint32_t key0, uint32_t key1, const uint32_t* ctr, uint32_t* out,
                         int64_t n, hipStream_t stream);
hipError_t launch_normals(uint32_t key0, uint32_t key1, const uint32_t* ctr, float* z, int64_t n,
                          hipStream_t stream);
// Solve grid of 8-state instances (vehicle = 1; persistent particles, no repair); x0_base holds
// 8 doubles per instance at x0_index.
hipError_t launch_solve8(const InstanceDesc* inst, const BlockDesc* blocks, int nblocks, int ppl,
                         size_t lds, const double* x0_base, int extra_shift, hipStream_t stream);
// one noise-free single-precision period of the 8-state vehicle: x[n][8], u[n][2] -> xn[n][8]
hipError_t launch_model_step8(const Car8F32& car, const float* x, const float* u, float* xn,
                              int64_t n, hipStream_t stream);

// disturbance words and normals of a solve through the solve kernel's path (lanes in {8, 16, 32,
// 64}, ppl in {1, 2, 4, 8}, lanes * ppl >= M)
hipError_t launch_disturbance(int lanes, int ppl, uint32_t key0, uint32_t key1, uint32_t s,
                              int K, int M, int T, int crn, float* w, uint32_t* words,
                              hipStream_t stream);
hipError_t launch_model_step(const CarF32& car, const float* x, const float* u, float* xn,
                             int64_t n, hipStream_t stream);
hipError_t launch_sdf(double a, double b, const double* pts, double* out, int64_t n,
                      hipStream_t stream);
hipError_t launch_repair(const ScoreF64& sc, const double* mom, const double* u_in, double* u_out,
                         int64_t n, hipStream_t stream);

}  // namespace bss
