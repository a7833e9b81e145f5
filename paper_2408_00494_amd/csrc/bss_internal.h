// bss_internal.h -- structures shared between the C ABI layer and the HIP kernels of libbssmppi.
//
// The rollout works in single precision on per-particle state; every per-(sample, step) scalar
// (moments, scores, the shield repair) and the K-reduction work in double precision.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace bss {

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

// Everything the double-precision per-(sample, step) code needs: model (for the shield's mean
// prediction), costs, barrier and repair settings.
struct ScoreF64 {
    double m, Iz, lf, lr, Cf, Cr, mu, g, v_min, dt;
    double steer_max, accel_max;
    double inv_var0, inv_var1;      // 1 / sigma_eps^2 (0 where the std is 0)
    double gamma_u, v_goal, q_vx, q_vy, q_r, q_ey, q_epsi, C_cbf, C_obs, phi_scale;
    double ell_a, ell_b, half_width;
    double nu, gamma, lambda;
    int32_t shield_iters;
    double shield_gmin, shield_fd;
};

// One solve's launch description.
struct SolveArgs {
    int32_t K, M, T;
    int32_t vshift;                // the mean sequence is read as v[min(t + vshift, T - 1)]
    uint32_t solve_index;
    uint32_t key0, key1;           // Philox key = (lo32 seed, hi32 seed)
    float steer_max, accel_max;
    float sig_eps0, sig_eps1;
    float sig_w0, sig_w1, sig_w2;
    CarF32 car;
    ScoreF64 sc;
    const double* x0;              // device [6]
    const double* Sigma0;          // device [36] row-major, or nullptr
    const double* v;               // device [T][2] mean sequence read by this solve
    float* u;                      // device [K][T][2] copy of the sampled controls, or nullptr
    double* mom;                   // device [K][T+1][9] beliefs (always written; scoring reads them)
    double* S;                     // device [K] trajectory costs
    double* partial;               // device [G][2T + 4] per-block log-sum-exp partials
};

// Per-block partial of the K-reduction (weights relative to the block's own minimum cost m_b):
//   [0, 2T)  N_i = sum_k w_k (u_{k,i} - v_i),   [2T] Z_b = sum w_k,   [2T+1] sum w_k^2,
//   [2T+2]   number of finite costs,            [2T+3] m_b (+inf if none is finite).
struct MergeArgs {
    int32_t T, G, vshift;
    double lambda;
    const double* partial;         // [G][2T + 4]
    const double* v_in;            // [T][2] mean sequence the solve read (with vshift)
    double* v_out;                 // [T][2] updated mean sequence (a different buffer)
    double* stats;                 // [8]: S_min, Z, ESS, #finite, status, v+_0 (2), unused
};

// samples per block of the partial kernel used for stand-alone K-reductions
constexpr int kPartialSlice = 16;

// lanes per sample (L) and particles per lane (P) of one rollout launch
struct LaunchShape {
    int lanes;
    int ppl;
};

constexpr int kMaxT = 256;
constexpr size_t kMaxLds = 65536;

// dynamic LDS of one solve block with L lanes per sample
size_t solve_lds_bytes(int lanes, int T);
LaunchShape choose_shape(int K, int M, int T, int requested_lanes);
int solve_blocks(int K, int lanes);

hipError_t launch_solve(const SolveArgs& a, LaunchShape shape, hipStream_t stream);
hipError_t launch_merge(const MergeArgs& a, hipStream_t stream);

// stand-alone kernels for staged checks
hipError_t launch_score(const SolveArgs& a, hipStream_t stream);
hipError_t launch_partials(int K, int T, double lambda, const double* S, const float* u,
                           const double* v, double* partial, hipStream_t stream);
int partial_blocks(int K);
hipError_t launch_philox(uint32_t key0, uint32_t key1, const uint32_t* ctr, uint32_t* out,
                         int64_t n, hipStream_t stream);
hipError_t launch_normals(uint32_t key0, uint32_t key1, const uint32_t* ctr, float* z, int64_t n,
                          hipStream_t stream);
hipError_t launch_model_step(const CarF32& car, const float* x, const float* u, float* xn,
                             int64_t n, hipStream_t stream);
hipError_t launch_sdf(double a, double b, const double* pts, double* out, int64_t n,
                      hipStream_t stream);
hipError_t launch_repair(const ScoreF64& sc, const double* mom, const double* u_in, double* u_out,
                         int64_t n, hipStream_t stream);

}  // namespace bss
