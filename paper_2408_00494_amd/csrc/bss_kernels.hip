// bss_kernels.hip -- HIP kernels of the BSS-MPPI solve for gfx950 (MI355X).
//
// One solve = two launches on one stream:
//   solve  : L lanes per control sample k (256/L samples per 256-thread block), P particles per
//            lane in registers.  Draws eps_{k,t} (Philox tag 0) lane-parallel over t, optionally
//            shield-repairs u_{k,t} per step, propagates the M particles with the single-
//            precision midpoint rule plus the disturbance (tag 1), reduces the particle mean and
//            position covariance across the L lanes in double precision every step (the belief
//            record of each step goes to a [K][T+1][9] buffer), then scores the belief
//            trajectory L records at a time (one per lane: signed distance, sigma_y, barrier h,
//            running cost, control cost, C_safe), and folds the block's samples into a
//            log-sum-exp partial (weights relative to the block's own minimum cost).  Scoring
//            after the particle loop keeps its double-precision temporaries out of the loop's
//            register budget.
//   merge  : one block per control entry (t, j): rescales the block partials to the global
//            minimum, exp(-(m_b - m)/lambda), and writes v+ = v + N/Z into the other buffer of the
//            ping-pong pair (so no block reads what another writes).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bss_device.h"
#include "bss_internal.h"

namespace bss {

namespace {

constexpr float kInv2Pi = 0.15915494309189535f;

__device__ __forceinline__ void kahan_add(float& s, float& c, float d)
{
    const float y = d - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Cholesky factor of the state-estimate covariance, per lane (6x6, semi-definite tolerated).
// Semi-definite factor for the Gaussian re-sampling draw: as chol6, but a pivot
// d <= 1e-10 A_jj + 1e-24 counts as zero (variances at the rounding level of an exactly degenerate
// particle set are not amplified).  Fully unrolled so that A and L stay in registers.
__device__ __forceinline__ void chol_psd6(const double (&A)[6][6], double (&L)[6][6])
{
#pragma unroll
    for (int j = 0; j < 6; ++j) {
#pragma unroll
        for (int i = 0; i < 6; ++i) L[i][j] = 0.0;
        double d = A[j][j];
#pragma unroll
        for (int q = 0; q < j; ++q) d -= L[j][q] * L[j][q];
        if (d > 1e-10 * A[j][j] + 1e-24) {
            const double ljj = sqrt(d);
            L[j][j] = ljj;
#pragma unroll
            for (int i = j + 1; i < 6; ++i) {
                double acc = A[i][j];
#pragma unroll
                for (int q = 0; q < j; ++q) acc -= L[i][q] * L[j][q];
                L[i][j] = acc / ljj;
            }
        }
    }
}

__device__ inline void chol6(const double* A, double* L)
{
    for (int i = 0; i < 36; ++i) L[i] = 0.0;
    for (int j = 0; j < 6; ++j) {
        double d = A[j * 6 + j];
        for (int q = 0; q < j; ++q) d -= L[j * 6 + q] * L[j * 6 + q];
        if (d <= 0.0) continue;
        const double ljj = sqrt(d);
        L[j * 6 + j] = ljj;
        for (int i = j + 1; i < 6; ++i) {
            double acc = A[i * 6 + j];
            for (int q = 0; q < j; ++q) acc -= L[i * 6 + q] * L[j * 6 + q];
            L[i * 6 + j] = acc / ljj;
        }
    }
}

// Cross-lane moves inside a row of 16 lanes (DPP): no LDS traffic, one VALU move per dword.  Every
// control used here reads a valid lane of the same row, so no "old" value is needed (bound_ctrl
// set): the destination register is not initialised first.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xf, 0xf, true));
}

constexpr int kDppQuadSwap1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kDppQuadSwap2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kDppHalfRowMirror = 0x141; // lane i <- lane 7-i within each 8
constexpr int kDppRowMirror = 0x140;     // lane i <- lane 15-i within each 16
constexpr int kDppRowBcast0 = 0x150;     // every lane of a row <- lane 0 of the row
constexpr int kDppRowBcast8 = 0x158;     // every lane of a row <- lane 8 of the row
constexpr int kDppQuadBcast0 = 0x00;     // quad_perm [0,0,0,0]
constexpr int kDppQuadBcast0And2 = 0xA0; // quad_perm [0,0,2,2]

// Cross-row exchanges with the gfx950 swap instructions (plain VALU ops, no LDS round trip).
// With both operands equal to x, v_permlane16_swap leaves in its first result, in every lane of
// a row pair (0,1) or (2,3), the even row's value of x and in its second result the odd row's;
// v_permlane32_swap does the same for the lower and upper halves of the wave.
__device__ __forceinline__ void pair_rows16(float x, float& even, float& odd)
{
    const uint32_t u = __float_as_uint(x);
    const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    even = __uint_as_float(r[0]);
    odd = __uint_as_float(r[1]);
}

__device__ __forceinline__ void pair_halves32(float x, float& lower, float& upper)
{
    const uint32_t u = __float_as_uint(x);
    const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    lower = __uint_as_float(r[0]);
    upper = __uint_as_float(r[1]);
}

__device__ __forceinline__ double xor16_sum(double x)
{
    const uint32_t lo = (uint32_t)__double2loint(x), hi = (uint32_t)__double2hiint(x);
    const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}

__device__ __forceinline__ double xor32_sum(double x)
{
    const uint32_t lo = (uint32_t)__double2loint(x), hi = (uint32_t)__double2hiint(x);
    const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}

// Sum over the L lanes of a group (L = 1, 2, 4, ..., 64, groups aligned in the wave, L uniform
// over the block), result in every lane of the group and bitwise identical across them (each
// stage adds the same two partial sums in either order).  Within a row of 16 the partners come
// from DPP; across rows from the swap instructions.
__device__ __forceinline__ double group_sum(double x, int L)
{
    if (L > 1) x += dpp_f64<kDppQuadSwap1>(x);
    if (L > 2) x += dpp_f64<kDppQuadSwap2>(x);
    if (L > 4) x += dpp_f64<kDppHalfRowMirror>(x);
    if (L > 8) x += dpp_f64<kDppRowMirror>(x);
    if (L > 16) x = xor16_sum(x);
    if (L > 32) x = xor32_sum(x);
    return x;
}

// Value of lane 0 of the group in every lane of the group.
__device__ __forceinline__ float group_first(float x, int L)
{
    if (L == 1) return x;
    if (L == 2) return dpp_f32<kDppQuadBcast0And2>(x);
    if (L == 4) return dpp_f32<kDppQuadBcast0>(x);
    if (L == 8) {
        const float a = dpp_f32<kDppRowBcast0>(x), b = dpp_f32<kDppRowBcast8>(x);
        return (threadIdx.x & 8) ? b : a;
    }
    float y = dpp_f32<kDppRowBcast0>(x);
    if (L == 16) return y;
    float even, odd;
    pair_rows16(y, even, odd);
    if (L == 32) return even;
    float lower, upper;
    pair_halves32(even, lower, upper);
    return lower;
}

__device__ __forceinline__ int vrow(int t, int vshift, int T)
{
    const int r = t + vshift;
    return r < T ? r : T - 1;
}

// Score one chunk of belief records, one record per lane of a W-lane group: running cost (times
// phi_scale on the terminal record), control cost on records < T, and C_safe on the transition
// into the record (record 0 has none).  `h_carry` holds h of the record before the chunk and is
// advanced to the chunk's last record.  Returns this lane's contribution.
// crec: the record's half-space constraint variances, or nullptr where the launch carries none.
__device__ inline double score_chunk(const ScoreF64& sc, const double* rec, int rec_idx, int count,
                                     int lane, int W, int T, const float2* u_row, const double* v,
                                     int vshift, double& h_carry, const double* crec = nullptr)
{
    const bool valid = lane < count;
    double part = 0.0;
    double h = 0.0;
    if (valid) {
        double scon[kMaxCon];
        if (crec) con_sigmas(sc, crec, scon);
        const BeliefEval be = eval_belief(sc, rec, crec ? scon : nullptr);
        double q = stage_cost(sc, rec, be);
        if (rec_idx == T) {
            q *= sc.phi_scale;
        } else {
            const float2 ut = u_row[rec_idx];
            const int r = vrow(rec_idx, vshift, T);
            q += sc.gamma_u * (v[2 * r] * sc.inv_var0 * (double)ut.x +
                               v[2 * r + 1] * sc.inv_var1 * (double)ut.y);
        }
        h = be.h;
        part = q;
    }
    const double h_left = __shfl(h, lane > 0 ? lane - 1 : 0, W);
    const double h_prev = lane == 0 ? h_carry : h_left;
    if (valid && rec_idx >= 1) part += sc.C_cbf * fmax(-h + (1.0 - sc.gamma) * h_prev, 0.0);
    h_carry = __shfl(h, count - 1, W);
    return part;
}

// Fold n samples (costs S_sh[0..n), controls u_sh[g][T]) into one log-sum-exp partial.
// Must be called by all 256 threads of the block after the inputs are visible in LDS.
__device__ inline void block_partial(int T, int n, const double* S_sh, double* w_sh,
                                     const float2* u_sh, const double* v, int vshift,
                                     double lambda, double* out)
{
    const int tid = threadIdx.x;
    double mb = INFINITY;
    for (int g = 0; g < n; ++g) {
        const double s = S_sh[g];
        if (isfinite(s)) mb = fmin(mb, s);
    }
    if (tid < n) {
        const double s = S_sh[tid];
        w_sh[tid] = (isfinite(s) && isfinite(mb)) ? exp(-(s - mb) / lambda) : 0.0;
    }
    __syncthreads();
    for (int i = tid; i < 2 * T; i += (int)blockDim.x) {
        const int t = i >> 1;
        const int r = vrow(t, vshift, T);
        const double vi = v[2 * r + (i & 1)];
        double acc = 0.0;
        for (int g = 0; g < n; ++g) {
            const float2 ut = u_sh[g * T + t];
            const double ui = (i & 1) ? (double)ut.y : (double)ut.x;
            acc += w_sh[g] * (ui - vi);
        }
        out[i] = acc;
    }
    if (tid == 0) {
        double Z = 0.0, W2 = 0.0, nf = 0.0;
        for (int g = 0; g < n; ++g) {
            Z += w_sh[g];
            W2 += w_sh[g] * w_sh[g];
            nf += isfinite(S_sh[g]) ? 1.0 : 0.0;
        }
        out[2 * T] = Z;
        out[2 * T + 1] = W2;
        out[2 * T + 2] = nf;
        out[2 * T + 3] = mb;
    }
}

// ----------------------------------------------------------------------------------------------
// solve: rollout + scoring + block partial of the K-reduction
// ----------------------------------------------------------------------------------------------
// Up to four particles per lane the loop fits 128 registers, which keeps four waves per SIMD;
// eight particles fit the budget of three, the shield's double-precision repair that of two.
// One solve block with L lanes per sample (L is a compile-time constant so that the group
// reductions are straight-line DPP sequences).
// Disturbance normals of step t for the P particles of one lane, written to slot t & 1 of the
// ring [2][P][3][256] (lane-contiguous, so the stores and the loads are conflict-free).
template <int P>
__device__ __forceinline__ void produce_noise(float* ring, int t, int q, const PhiloxParticle* pp,
                                              uint32_t c3w, uint32_t lk, uint32_t key0,
                                              uint32_t key1)
{
    const PhiloxStep ps = philox_step((uint32_t)t, c3w, lk, key0, key1);
    float* dst = ring + (t & 1) * (P * 3 * 256) + q;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        uint32_t c0, c1, c2, c3;
        philox10_tail(ps, pp[p], key0, key1, c0, c1, c2, c3);
        float w0, w1;
        bm_pair(c0, c1, w0, w1);
        dst[(p * 3 + 0) * 256] = w0;
        dst[(p * 3 + 1) * 256] = w1;
        dst[(p * 3 + 2) * 256] = bm_cos(c2, c3);
    }
}

// Gaussian re-sampling of Alg. 2 as printed: the particles of step t are redrawn as
// xbar_t + L_t xi with xbar_t and the unbiased full 6x6 covariance of the current set of the
// sample (FP64 group sums of the components shifted by particle 0: 6 sums and 21 products) and
// L_t its semi-definite factor; xi are six standard normals from tags 4 and 5 with counter
// (t, m, k).  Positions and heading stay compensated pairs relative to the estimate.
//
// Sigma points (mode 2, M = 12): the same moments with equal weights 1/12, plus the disturbance
// covariance diag(0, 0, 0, sigma_w^2) scaled by qbar (the previous points' mean of
// (1 + kappa |vx|)^2), and the deterministic points mean +- sqrt(6) L e_i instead of the draw.
template <int P, int L>
__device__ __forceinline__ void resample_particles(int t, int j, int k, int M, uint32_t s,
                                                   uint32_t key0, uint32_t key1, int mode,
                                                   double qbar, const float* sw, float* Xs,
                                                   float* Xc, float* Ys, float* Yc, float* Ps,
                                                   float* Pc, float* vx, float* vy, float* vr)
{
    double ref[6];
    ref[0] = (double)group_first(Xs[0], L) - (double)group_first(Xc[0], L);
    ref[1] = (double)group_first(Ys[0], L) - (double)group_first(Yc[0], L);
    ref[2] = (double)group_first(Ps[0], L) - (double)group_first(Pc[0], L);
    ref[3] = (double)group_first(vx[0], L);
    ref[4] = (double)group_first(vy[0], L);
    ref[5] = (double)group_first(vr[0], L);
    double sd[6], sq[6][6];
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        sd[a] = 0.0;
#pragma unroll
        for (int b = 0; b <= a; ++b) sq[a][b] = 0.0;
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (j + p * L < M) {
            double dv[6];
            dv[0] = ((double)Xs[p] - (double)Xc[p]) - ref[0];
            dv[1] = ((double)Ys[p] - (double)Yc[p]) - ref[1];
            dv[2] = ((double)Ps[p] - (double)Pc[p]) - ref[2];
            dv[3] = (double)vx[p] - ref[3];
            dv[4] = (double)vy[p] - ref[4];
            dv[5] = (double)vr[p] - ref[5];
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                sd[a] += dv[a];
#pragma unroll
                for (int b = 0; b <= a; ++b) sq[a][b] = fma(dv[a], dv[b], sq[a][b]);
            }
        }
    }
    const double invM = 1.0 / (double)M;
    const double invM1 = mode == 2 ? invM : (M > 1 ? 1.0 / (double)(M - 1) : 0.0);
    double mean[6], cov[6][6];
#pragma unroll
    for (int a = 0; a < 6; ++a) sd[a] = group_sum(sd[a], L);
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        mean[a] = ref[a] + sd[a] * invM;
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const double c = (group_sum(sq[a][b], L) - sd[a] * (sd[b] * invM)) * invM1;
            cov[a][b] = c;
            cov[b][a] = c;
        }
    }
    if (mode == 2) {
#pragma unroll
        for (int a = 0; a < 3; ++a) cov[3 + a][3 + a] += (double)sw[a] * (double)sw[a] * qbar;
    }
    double Lf[6][6];
    chol_psd6(cov, Lf);
    const uint32_t c3a = rng_word3(kTagResample0, s), c3b = rng_word3(kTagResample1, s);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint32_t m = (uint32_t)(j + p * L);
        double xi[6];
        if (mode == 2) {
            // selects instead of a runtime index keep xi in registers
            const double r = m < 6u ? 2.449489742783178 : -2.449489742783178;
            const uint32_t e = m % 6u;
#pragma unroll
            for (int a = 0; a < 6; ++a) xi[a] = (m < 12u && e == (uint32_t)a) ? r : 0.0;
        } else {
#pragma unroll
            for (int blk = 0; blk < 2; ++blk) {
                uint32_t c0 = (uint32_t)t, c1 = m, c2 = (uint32_t)k, c3 = blk ? c3b : c3a;
                philox10(c0, c1, c2, c3, key0, key1);
                float z0, z1;
                bm_pair(c0, c1, z0, z1);
                xi[3 * blk + 0] = z0;
                xi[3 * blk + 1] = z1;
                xi[3 * blk + 2] = bm_cos(c2, c3);
            }
        }
        double dev[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            double acc = mean[a];
#pragma unroll
            for (int b = 0; b <= a; ++b) acc = fma(Lf[a][b], xi[b], acc);
            dev[a] = acc;
        }
        Xs[p] = (float)dev[0];
        Xc[p] = (float)((double)Xs[p] - dev[0]);
        Ys[p] = (float)dev[1];
        Yc[p] = (float)((double)Ys[p] - dev[1]);
        Ps[p] = (float)dev[2];
        Pc[p] = (float)((double)Ps[p] - dev[2]);
        vx[p] = (float)dev[3];
        vy[p] = (float)dev[4];
        vr[p] = (float)dev[5];
    }
}

// One solve block with L lanes per sample (L is a compile-time constant so that the group
// reductions are straight-line DPP sequences).
//
// SPLIT (512 threads): threads 256..511 generate the disturbance normals of step t + 1 while
// threads 0..255 integrate step t, through a two-slot LDS ring and one barrier per step.  This
// puts two waves on every SIMD when a launch has too few samples to fill the chip otherwise (a
// lone wave issues at about half the SIMD's rate); the arithmetic and its order are unchanged, so
// the results are bitwise the same as without the split.
template <int P, bool SHIELD, int L, bool SPLIT, bool RESAMPLE, bool CON>
__device__ __forceinline__ void solve_block(const InstanceDesc& d, const BlockDesc bd,
                                            const double* __restrict__ x0_base,
                                            const double* __restrict__ Sigma0_base,
                                            int extra_shift)
{
    static_assert(!(SPLIT && SHIELD), "the shielded loop is not split");
    static_assert(!(SPLIT && RESAMPLE), "the re-sampling loop is not split");
    static_assert(!CON || (SHIELD && RESAMPLE && !SPLIT) || (!SHIELD && !RESAMPLE),
                  "half-space constraints: the plain, split and generic variants only");
    constexpr int log2L = L == 8 ? 3 : (L == 16 ? 4 : (L == 32 ? 5 : 6));
    constexpr int groups = 256 >> log2L;
    const int T = d.T, M = d.M;
    const int vshift = d.vshift + extra_shift;
    const double* __restrict__ v = d.v[d.cur];
    extern __shared__ double smem[];
    double* S_sh = smem;                                     // [groups]
    double* w_sh = S_sh + groups;                            // [groups]
    float2* u_sh = reinterpret_cast<float2*>(w_sh + groups);  // [groups][T]
    float* ring = reinterpret_cast<float*>(u_sh + groups * T);  // SPLIT: [2][P][3][256]
    const int q = SPLIT ? (int)(threadIdx.x & 255u) : (int)threadIdx.x;
    const bool producer = SPLIT && threadIdx.x >= 256u;
    const int g = q >> log2L;
    const int j = q & (L - 1);
    const int k = bd.k0 + g;
    const bool active = k < d.K;
    float2* us = u_sh + g * T;
    double* mom_k = d.mom + (size_t)(active ? k : 0) * (T + 1) * 9;
    const uint32_t s = d.solve_index;
    const uint32_t key0 = d.key0, key1 = d.key1;
    const double* x0p = x0_base + 6 * d.x0_index;
    const double* S0p = Sigma0_base ? Sigma0_base + 36 * d.x0_index : nullptr;
    // half-space constraints on the whole state (compiled into the CON variants only): their
    // variances a_i^T Sigma a_i per record
    const int ncon = CON ? d.sc.n_con : 0;
    double* cvar_k = ncon > 0 ? d.cvar + (size_t)(active ? k : 0) * (T + 1) * ncon : nullptr;

    // ---- phase 1: control samples u_{k,t} = clip(v_t + eps_{k,t}), lane-parallel over t ----
    if (active && (!SPLIT || producer)) {
        const float sig0 = d.sig_eps0, sig1 = d.sig_eps1;
        const float smax = d.steer_max, amax = d.accel_max;
        for (int t = j; t < T; t += L) {
            uint32_t c0 = (uint32_t)t, c1 = 0u, c2 = (uint32_t)k, c3 = rng_word3(kTagEps, s);
            philox10(c0, c1, c2, c3, key0, key1);
            float z0, z1;
            bm_pair(c0, c1, z0, z1);
            const int r = vrow(t, vshift, T);
            const float v0 = (float)v[2 * r], v1 = (float)v[2 * r + 1];
            const float u0 = fminf(fmaxf(fmaf(sig0, z0, v0), -smax), smax);
            const float u1 = fminf(fmaxf(fmaf(sig1, z1, v1), -amax), amax);
            us[t] = make_float2(u0, u1);
            if (!SHIELD && d.u) reinterpret_cast<float2*>(d.u)[(size_t)k * T + t] = us[t];
        }
    }
    // disturbance stream of this lane's particles: the first two Philox rounds are partly shared;
    // with common random numbers every sample draws the stream of sample word 0
    const uint32_t c3w = rng_word3(kTagW, s);
    const uint64_t pk = (uint64_t)kPhiloxM1 * (d.crn ? 0u : (uint32_t)k);
    const uint32_t hk = (uint32_t)(pk >> 32), lk = (uint32_t)pk;
    if (SPLIT && producer && active) {
        PhiloxParticle pp0[P];
#pragma unroll
        for (int p = 0; p < P; ++p) pp0[p] = philox_particle((uint32_t)(j + p * L), hk, key0, key1);
        produce_noise<P>(ring, 0, q, pp0, c3w, lk, key0, key1);
    }
    __syncthreads();

    if (SPLIT || active) {
        const bool consumer = !producer && active;
        double x0[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) x0[i] = x0p[i];
        const bool spread = S0p != nullptr;

        // state relative to the estimate: position and heading as compensated (sum, correction)
        float Xs[P], Xc[P], Ys[P], Yc[P], Ps[P], Pc[P], vx[P], vy[P], vr[P];
        if (consumer) {
            double L0[36];
            if (spread) chol6(S0p, L0);
            // sigma points at t = 0: mean +- sqrt(6) L e_i of the given estimate
            const bool sigma = RESAMPLE && d.belief == 2;
            double Lp[6][6];
            if (sigma) {
                double A[6][6];
#pragma unroll
                for (int a = 0; a < 6; ++a)
#pragma unroll
                    for (int b = 0; b < 6; ++b) A[a][b] = spread ? S0p[a * 6 + b] : 0.0;
                chol_psd6(A, Lp);
            }
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int m = j + p * L;
                double dev[6] = {0, 0, 0, 0, 0, 0};
                if (sigma) {
                    const double r = m < 6 ? 2.449489742783178 : -2.449489742783178;
                    const int e = m % 6;
#pragma unroll
                    for (int a = 0; a < 6; ++a) {
                        double acc = 0.0;
#pragma unroll
                        for (int b = 0; b < 6; ++b) acc = (m < 12 && e == b) ? r * Lp[a][b] : acc;
                        dev[a] = acc;
                    }
                } else if (spread) {
                    double xi[6];
#pragma unroll
                    for (int blk = 0; blk < 2; ++blk) {
                        uint32_t c0 = (uint32_t)blk, c1 = (uint32_t)m, c2 = (uint32_t)k,
                                 c3 = rng_word3(kTagInit, s);
                        philox10(c0, c1, c2, c3, key0, key1);
                        float z0, z1;
                        bm_pair(c0, c1, z0, z1);
                        xi[blk * 3 + 0] = z0;
                        xi[blk * 3 + 1] = z1;
                        xi[blk * 3 + 2] = bm_cos(c2, c3);
                    }
                    for (int i = 0; i < 6; ++i) {
                        double acc = 0.0;
                        for (int q = 0; q <= i; ++q) acc += L0[i * 6 + q] * xi[q];
                        dev[i] = acc;
                    }
                }
                Xs[p] = (float)dev[0];
                Xc[p] = (float)((double)Xs[p] - dev[0]);
                Ys[p] = (float)dev[1];
                Yc[p] = (float)((double)Ys[p] - dev[1]);
                Ps[p] = (float)dev[2];
                Pc[p] = (float)((double)Ps[p] - dev[2]);
                vx[p] = (float)(x0[3] + dev[3]);
                vy[p] = (float)(x0[4] + dev[4]);
                vr[p] = (float)(x0[5] + dev[5]);
            }
        }
        const double rev0d = x0[2] * 0.15915494309189535;
        const float rev0 = (float)(rev0d - rint(rev0d));
        const CarF32 car = d.car;
        const float sw0 = d.sig_w0, sw1 = d.sig_w1, sw2 = d.sig_w2;
        const float ksp = d.sig_w_speed;

        // belief at t = 0 is the given estimate (record 0)
        double bel[9];
#pragma unroll
        for (int i = 0; i < 6; ++i) bel[i] = x0[i];
        bel[6] = spread ? S0p[0] : 0.0;
        bel[7] = spread ? S0p[1] : 0.0;
        bel[8] = spread ? S0p[7] : 0.0;
        // a_i^T Sigma a_i of each half-space constraint (eq. 11 with eta_i = a_i); at t = 0 from
        // the given covariance
        double bcv[kMaxCon];
#pragma unroll
        for (int c = 0; c < kMaxCon; ++c) {
            double q = 0.0;
            if (c < ncon && spread) {
                const double* a = d.sc.con_a + 6 * c;
                for (int r = 0; r < 6; ++r) {
                    double row = 0.0;
                    for (int e = 0; e < 6; ++e) row = fma(S0p[r * 6 + e], a[e], row);
                    q = fma(a[r], row, q);
                }
            }
            bcv[c] = q;
        }
        if (consumer && j == 0) {
#pragma unroll
            for (int i = 0; i < 9; ++i) mom_k[i] = bel[i];
#pragma unroll
            for (int c = 0; c < kMaxCon; ++c)
                if (c < ncon) cvar_k[c] = bcv[c];
        }
        PhiloxParticle pp[P];
#pragma unroll
        for (int p = 0; p < P; ++p) pp[p] = philox_particle((uint32_t)(j + p * L), hk, key0, key1);
        const double invM = 1.0 / (double)M;
        const double invM1 =
            (RESAMPLE && d.belief == 2) ? invM : (M > 1 ? 1.0 / (double)(M - 1) : 0.0);
        const float swv[3] = {sw0, sw1, sw2};
        double qbar = 1.0;      // sigma points: previous points' mean of (1 + kappa |vx|)^2

        // In split mode every thread runs every iteration and meets exactly one barrier per step,
        // outside all divergent branches (waves may hold both active and inactive samples).
        for (int t = 0; t < T; ++t) {
            if (SPLIT && producer) {
                if (active && t + 1 < T) produce_noise<P>(ring, t + 1, q, pp, c3w, lk, key0, key1);
            } else if (!SPLIT || consumer) {
                float2 uu = us[t];
                if (SHIELD) {
                    const ScoreF64& sc = d.sc;
                    if (sc.shield_iters > 0) {
                        double scon[kMaxCon];
                        if (ncon > 0) con_sigmas(sc, bcv, scon);
                        const double* sc_con = ncon > 0 ? scon : nullptr;
                        const BeliefEval be = eval_belief(sc, bel, sc_con);
                        const double fd = sc.shield_fd;
                        const int role = j < 5 ? j : 0;
                        const double o0 = role == 1 ? fd : (role == 2 ? -fd : 0.0);
                        const double o1 = role == 3 ? fd : (role == 4 ? -fd : 0.0);
                        double us0 = uu.x, us1 = uu.y;
                        for (int it = 0; it < sc.shield_iters; ++it) {
                            // lanes 0-4 of the group evaluate r at u and at the four
                            // difference points
                            const double rv = repair_residual(sc, bel, be, be.h, us0 + o0,
                                                              us1 + o1, sc_con);
                            const double r0 = __shfl(rv, 0, L);
                            const double rp0 = __shfl(rv, 1, L), rm0 = __shfl(rv, 2, L);
                            const double rp1 = __shfl(rv, 3, L), rm1 = __shfl(rv, 4, L);
                            if (!(r0 > 0.0)) break;
                            const double g0 = (rp0 - rm0) / (2.0 * fd);
                            const double g1 = (rp1 - rm1) / (2.0 * fd);
                            const double den = g0 * g0 + g1 * g1 + sc.shield_gmin * sc.shield_gmin;
                            us0 = clampd(us0 - r0 * g0 / den, -sc.steer_max, sc.steer_max);
                            us1 = clampd(us1 - r0 * g1 / den, -sc.accel_max, sc.accel_max);
                        }
                        uu = make_float2((float)us0, (float)us1);
                    }
                    if (j == 0) {
                        us[t] = uu;
                        if (d.u) reinterpret_cast<float2*>(d.u)[(size_t)k * T + t] = uu;
                    }
                }
                if (RESAMPLE && d.belief != 0 && t > 0)
                    resample_particles<P, L>(t, j, k, M, s, key0, key1, d.belief, qbar, swv, Xs,
                                             Xc, Ys, Yc, Ps, Pc, vx, vy, vr);
                if (RESAMPLE && d.belief == 2) {
                    double qs = 0.0;
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        if (j + p * L < M) {
                            const double f = 1.0 + (double)ksp * fabs((double)vx[p]);
                            qs = fma(f, f, qs);
                        }
                    }
                    qbar = group_sum(qs, L) * invM;
                }
                const StepF32 st = make_step(car, uu.x, uu.y);
                PhiloxStep ps{};
                if (!SPLIT) ps = philox_step((uint32_t)t, c3w, lk, key0, key1);
                // FP64 moment sums of the lane's particles; positions shifted by particle 0 of
                // the sample (lane 0 of the group), taken after its update in the first chunk
                double sX = 0, sY = 0, sP = 0, svx = 0, svy = 0, svr = 0, sXX = 0, sXY = 0,
                       sYY = 0;
                double refX = 0.0, refY = 0.0;
                // sums of squares of the constraint projections y = a_i^T (x - xref), xref the
                // estimate with particle 0's position (the sums of y follow from the moment sums)
                double c2[kMaxCon];
#pragma unroll
                for (int c = 0; c < kMaxCon; ++c) c2[c] = 0.0;
                // With up to four particles per lane the step runs in stages over all of them
                // (disturbance normals, first field evaluation, midpoint, second evaluation,
                // update), each stage one straight-line block with no per-particle branch, so
                // that the compiler interleaves the particles' independent dependency chains.
                // With eight, the staged form does not fit the registers of three waves per
                // SIMD; those particles are stepped one after the other (several waves per SIMD
                // hide the latency instead), except in the repair's variant, whose two waves per
                // SIMD leave room for stages over four particles at a time.
                constexpr int Q = P <= 4 ? P : (SHIELD && !RESAMPLE && !CON ? 4 : 1);
#pragma unroll
                for (int p0 = 0; p0 < P; p0 += Q) {
                    float w0[Q], w1[Q], w2[Q];
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        const int p = p0 + i;
                        if (RESAMPLE && d.belief == 2) {
                            w0[i] = w1[i] = w2[i] = 0.0f;   // sigma points: Q enters instead
                        } else if (SPLIT) {
                            const float* src = ring + (t & 1) * (P * 3 * 256) + q;
                            w0[i] = src[(p * 3 + 0) * 256];
                            w1[i] = src[(p * 3 + 1) * 256];
                            w2[i] = src[(p * 3 + 2) * 256];
                        } else {
                            uint32_t c0, c1, c2, c3;
                            philox10_tail(ps, pp[p], key0, key1, c0, c1, c2, c3);
                            bm_pair(c0, c1, w0[i], w1[i]);
                            w2[i] = bm_cos(c2, c3);
                        }
                    }
                    if (ksp != 0.0f) {
                        // state-dependent disturbance: std sigma_w (1 + kappa |vx|) at the
                        // step's starting state
#pragma unroll
                        for (int i = 0; i < Q; ++i) {
                            const float fw = fmaf(ksp, fabsf(vx[p0 + i]), 1.0f);
                            w0[i] *= fw;
                            w1[i] *= fw;
                            w2[i] *= fw;
                        }
                    }
                    float rev[Q], dX[Q], dY[Q], dvx[Q], dvy[Q], dr[Q];
                    float vxm[Q], vym[Q], vrm[Q];
#pragma unroll
                    for (int i = 0; i < Q; ++i) rev[i] = fmaf(Ps[p0 + i], kInv2Pi, rev0);
                    car_field_f32_n<Q>(car, st, rev, vx + p0, vy + p0, vr + p0, dX, dY, dvx, dvy,
                                       dr);
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        const int p = p0 + i;
                        rev[i] = fmaf(fmaf(car.half_dt, vr[p], Ps[p]), kInv2Pi, rev0);
                        vxm[i] = fmaf(car.half_dt, dvx[i], vx[p]);
                        vym[i] = fmaf(car.half_dt, dvy[i], vy[p]);
                        vrm[i] = fmaf(car.half_dt, dr[i], vr[p]);
                    }
                    car_field_f32_n<Q>(car, st, rev, vxm, vym, vrm, dX, dY, dvx, dvy, dr);
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        const int p = p0 + i;
                        kahan_add(Xs[p], Xc[p], car.dt * dX[i]);
                        kahan_add(Ys[p], Yc[p], car.dt * dY[i]);
                        kahan_add(Ps[p], Pc[p], car.dt * vrm[i]);
                        vx[p] = fmaf(sw0, w0[i], fmaf(car.dt, dvx[i], vx[p]));
                        vy[p] = fmaf(sw1, w1[i], fmaf(car.dt, dvy[i], vy[p]));
                        vr[p] = fmaf(sw2, w2[i], fmaf(car.dt, dr[i], vr[p]));
                    }
                    if (p0 == 0) {
                        refX = (double)group_first(Xs[0], L) - (double)group_first(Xc[0], L);
                        refY = (double)group_first(Ys[0], L) - (double)group_first(Yc[0], L);
                    }
                    // accumulate the chunk (particles beyond M contribute nothing)
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        const int p = p0 + i;
                        if (j + p * L < M) {
                            const double X = ((double)Xs[p] - (double)Xc[p]) - refX;
                            const double Y = ((double)Ys[p] - (double)Yc[p]) - refY;
                            sX += X;
                            sY += Y;
                            sP += (double)Ps[p] - (double)Pc[p];
                            svx += (double)vx[p];
                            svy += (double)vy[p];
                            svr += (double)vr[p];
                            sXX = fma(X, X, sXX);
                            sXY = fma(X, Y, sXY);
                            sYY = fma(Y, Y, sYY);
#pragma unroll
                            for (int c = 0; c < kMaxCon; ++c) {
                                if (c < ncon) {
                                    const double* a = d.sc.con_a + 6 * c;
                                    const double y = fma(
                                        a[0], X,
                                        fma(a[1], Y,
                                            fma(a[2], (double)Ps[p] - (double)Pc[p],
                                                fma(a[3], (double)vx[p] - x0[3],
                                                    fma(a[4], (double)vy[p] - x0[4],
                                                        a[5] * ((double)vr[p] - x0[5]))))));
                                    c2[c] = fma(y, y, c2[c]);
                                }
                            }
                        }
                    }
                }
                // moments: FP64 sums over the L lanes (DPP inside a row, swaps across rows)
                sX = group_sum(sX, L);
                sY = group_sum(sY, L);
                sP = group_sum(sP, L);
                svx = group_sum(svx, L);
                svy = group_sum(svy, L);
                svr = group_sum(svr, L);
                sXX = group_sum(sXX, L);
                sXY = group_sum(sXY, L);
                sYY = group_sum(sYY, L);
                const double mX = sX * invM, mY = sY * invM;
                bel[0] = x0[0] + (refX + mX);
                bel[1] = x0[1] + (refY + mY);
                bel[2] = x0[2] + sP * invM;
                bel[3] = svx * invM;
                bel[4] = svy * invM;
                bel[5] = svr * invM;
                bel[6] = (sXX - sX * mX) * invM1;
                bel[7] = (sXY - sX * mY) * invM1;
                bel[8] = (sYY - sY * mY) * invM1;
#pragma unroll
                for (int c = 0; c < kMaxCon; ++c) {
                    if (c < ncon) {
                        // sum of the projections from the moment sums, then the unbiased variance
                        const double* a = d.sc.con_a + 6 * c;
                        const double s1 =
                            fma(a[0], sX,
                                fma(a[1], sY,
                                    fma(a[2], sP,
                                        fma(a[3], fma(-(double)M, x0[3], svx),
                                            fma(a[4], fma(-(double)M, x0[4], svy),
                                                a[5] * fma(-(double)M, x0[5], svr))))));
                        const double s2 = group_sum(c2[c], L);
                        double var = (s2 - s1 * (s1 * invM)) * invM1;
                        if (d.belief == 2) {
                            // sigma points: plus a_i^T Q a_i of the disturbance covariance,
                            // scaled like Q by the points' mean of (1 + kappa |vx|)^2
                            const double q0 = a[3] * (double)sw0, q1 = a[4] * (double)sw1,
                                         q2 = a[5] * (double)sw2;
                            var = fma(qbar, fma(q0, q0, fma(q1, q1, q2 * q2)), var);
                        }
                        bcv[c] = var;
                    }
                }

                // record t+1, written by lane (t+1) % L of the group (spreads the stores)
                if (j == ((t + 1) & (L - 1))) {
                    double* rec = mom_k + (size_t)(t + 1) * 9;
#pragma unroll
                    for (int i = 0; i < 9; ++i) rec[i] = bel[i];
#pragma unroll
                    for (int c = 0; c < kMaxCon; ++c)
                        if (c < ncon) cvar_k[(size_t)(t + 1) * ncon + c] = bcv[c];
                }
            }
            if (SPLIT) __syncthreads();
        }
    }
    // ---- phase 3: score the belief trajectory, L records at a time (one per lane) ----
    __threadfence_block();
    __syncthreads();
    double S_part = 0.0;
    if (active && !producer) {
        double h_carry = 0.0;
        for (int base = 0; base <= T; base += L) {
            const int count = min(L, T + 1 - base);
            const int rec = base + min(j, count - 1);
            S_part += score_chunk(d.sc, mom_k + (size_t)rec * 9, base + j, count, j, L, T, us, v,
                                  vshift, h_carry,
                                  ncon > 0 ? cvar_k + (size_t)rec * ncon : nullptr);
        }
    }
    const double S_k = group_sum(S_part, L);
    if (j == 0 && !producer) {
        S_sh[g] = active ? S_k : INFINITY;
        if (active) d.S[k] = S_k;
    }
    __syncthreads();
    const int n = min(groups, d.K - bd.k0);
    block_partial(T, n, S_sh, w_sh, u_sh, v, vshift, d.sc.lambda,
                  d.partial + (size_t)(bd.k0 >> (8 - log2L)) * (2 * T + 4));
}

// Solve grid: every block looks up its instance and first sample; the lane count is uniform over
// a block, so the dispatch below is a block-uniform branch.
template <int P, bool SHIELD, bool SPLIT, bool RESAMPLE, bool CON = false>
__global__ __launch_bounds__(SPLIT ? 512 : 256)
__attribute__((amdgpu_waves_per_eu((SHIELD || RESAMPLE || CON) ? 2
                                   : (P <= 4 ? (SPLIT ? 2 : 4) : 3)))) void solve_kernel(
    const InstanceDesc* __restrict__ insts, const BlockDesc* __restrict__ blocks,
    const double* __restrict__ x0_base, const double* __restrict__ Sigma0_base, int extra_shift)
{
    const BlockDesc bd = blocks[blockIdx.x];
    const InstanceDesc& d = insts[bd.inst];
    switch (d.lanes) {
    case 8:
        solve_block<P, SHIELD, 8, SPLIT, RESAMPLE, CON>(d, bd, x0_base, Sigma0_base, extra_shift);
        break;
    case 16:
        solve_block<P, SHIELD, 16, SPLIT, RESAMPLE, CON>(d, bd, x0_base, Sigma0_base, extra_shift);
        break;
    case 32:
        solve_block<P, SHIELD, 32, SPLIT, RESAMPLE, CON>(d, bd, x0_base, Sigma0_base, extra_shift);
        break;
    default:
        solve_block<P, SHIELD, 64, SPLIT, RESAMPLE, CON>(d, bd, x0_base, Sigma0_base, extra_shift);
        break;
    }
}

// ----------------------------------------------------------------------------------------------
// merge: one block per control entry
// ----------------------------------------------------------------------------------------------
// Reduction over the 64 lanes of a wave (DPP within rows, swaps across rows); every lane gets the
// result, bitwise identical across lanes (each stage combines the same two values).
struct MinOp {
    __device__ double operator()(double a, double b) const { return fmin(a, b); }
};
struct AddOp {
    __device__ double operator()(double a, double b) const { return a + b; }
};

template <class Op>
__device__ __forceinline__ double wave_reduce(double x, Op op)
{
    x = op(x, dpp_f64<kDppQuadSwap1>(x));
    x = op(x, dpp_f64<kDppQuadSwap2>(x));
    x = op(x, dpp_f64<kDppHalfRowMirror>(x));
    x = op(x, dpp_f64<kDppRowMirror>(x));
    {
        const uint32_t lo = (uint32_t)__double2loint(x), hi = (uint32_t)__double2hiint(x);
        const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        x = op(__hiloint2double((int)b[0], (int)a[0]), __hiloint2double((int)b[1], (int)a[1]));
    }
    {
        const uint32_t lo = (uint32_t)__double2loint(x), hi = (uint32_t)__double2hiint(x);
        const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        x = op(__hiloint2double((int)b[0], (int)a[0]), __hiloint2double((int)b[1], (int)a[1]));
    }
    return x;
}

// Merge of one control entry by one wave: global minimum m = min_b m_b, rescale
// exp(-(m_b - m)/lambda), fixed-order reductions of Z, sum w^2, #finite and the entry's numerator
// (lane l takes blocks l, l + 64, ...); results in every lane.
__device__ inline void merge_entry(const double* partial, int G, int T, int col, double lambda,
                                   double& m, double& Z, double& W2, double& nf, double& N)
{
    const int lane = (int)(threadIdx.x & 63u);
    const int stride = 2 * T + 4;
    // up to four blocks per lane are loaded in one pass (all loads in flight together); larger
    // grids fall back to a second pass over the remaining blocks
    constexpr int kHeld = 4;
    double hm[kHeld], hz[kHeld], hw[kHeld], hn[kHeld], hc[kHeld];
#pragma unroll
    for (int i = 0; i < kHeld; ++i) {
        const int b = lane + 64 * i;
        const double* pb = partial + (size_t)(b < G ? b : 0) * stride;
        hm[i] = b < G ? pb[2 * T + 3] : INFINITY;
        hz[i] = b < G ? pb[2 * T] : 0.0;
        hw[i] = b < G ? pb[2 * T + 1] : 0.0;
        hn[i] = b < G ? pb[2 * T + 2] : 0.0;
        hc[i] = b < G ? pb[col] : 0.0;
    }
    m = INFINITY;
#pragma unroll
    for (int i = 0; i < kHeld; ++i) m = fmin(m, hm[i]);
    for (int b = lane + 64 * kHeld; b < G; b += 64)
        m = fmin(m, partial[(size_t)b * stride + 2 * T + 3]);
    m = wave_reduce(m, MinOp());
    Z = 0.0;
    W2 = 0.0;
    nf = 0.0;
    N = 0.0;
#pragma unroll
    for (int i = 0; i < kHeld; ++i) {
        const double sc = isfinite(hm[i]) ? exp(-(hm[i] - m) / lambda) : 0.0;
        Z += sc * hz[i];
        W2 += sc * sc * hw[i];
        nf += hn[i];
        N += sc * hc[i];
    }
    for (int b = lane + 64 * kHeld; b < G; b += 64) {
        const double* pb = partial + (size_t)b * stride;
        const double mb = pb[2 * T + 3];
        const double sc = isfinite(mb) ? exp(-(mb - m) / lambda) : 0.0;
        Z += sc * pb[2 * T];
        W2 += sc * sc * pb[2 * T + 1];
        nf += pb[2 * T + 2];
        N += sc * pb[col];
    }
    Z = wave_reduce(Z, AddOp());
    W2 = wave_reduce(W2, AddOp());
    nf = wave_reduce(nf, AddOp());
    N = wave_reduce(N, AddOp());
}

__device__ inline void write_stats(double* stats, int col, double vo, bool ok, double m, double Z,
                                   double W2, double nf)
{
    if (col < 2) stats[5 + col] = vo;
    if (col == 0) {
        stats[0] = m;
        stats[1] = Z;
        stats[2] = ok ? Z * Z / W2 : 0.0;
        stats[3] = nf;
        stats[4] = ok ? 0.0 : 5.0;
        stats[7] = 0.0;
    }
}

// One wave per (instance, control entry), four per block.  v+ goes to the other buffer of the
// instance's ping-pong pair; the last wave of an instance to finish advances its per-solve state.
// Nothing in this launch reads what the others write (the counter only elects the last wave; v+,
// the statistics and the state are read by later launches, which the launch boundary orders), so
// no fence is issued: a device-scope release writes back the chip-level cache.
__global__ __launch_bounds__(256) void merge_kernel(InstanceDesc* insts, const MergeDesc* cols,
                                                    int ncols, int extra_shift)
{
    const int idx = (int)(blockIdx.x * 4u + (threadIdx.x >> 6));
    if (idx >= ncols) return;
    const MergeDesc md = cols[idx];
    InstanceDesc& d = insts[md.inst];
    const int T = d.T, col = md.col;
    const int cur = d.cur;
    // the entry's current mean value is loaded before the reduction so the load overlaps it
    const int r = vrow(col >> 1, d.vshift + extra_shift, T);
    const double vi = d.v[cur][2 * r + (col & 1)];
    double m, Z, W2, nf, N;
    merge_entry(d.partial, d.nblocks, T, col, d.sc.lambda, m, Z, W2, nf, N);
    if ((threadIdx.x & 63u) == 0) {
        const bool ok = nf > 0.0 && Z > 0.0;
        const double vo = ok ? vi + N / Z : vi;
        d.v[1 - cur][col] = vo;
        write_stats(d.stats, col, vo, ok, m, Z, W2, nf);
        const uint32_t prev = atomicAdd(&d.done, 1u);
        if (prev == (uint32_t)(2 * T - 1)) {
            // every entry of this instance is written: publish the new state
            d.done = 0u;
            d.cur = 1 - cur;
            d.vshift = d.shift_after;
            d.solve_index = d.solve_index + 1u;
            d.status = ok ? 0 : 5;
        }
    }
}

// Repair of the updated sequence (local repair of v+): the repair descriptor is a copy of the
// instance's with one sample, no exploration noise, its own Philox key and its own buffers, and
// both mean-sequence pointers of the instance.  Before its rollout it takes the instance's state
// as the merge left it: the buffer holding v+, no pending shift (v+ is read as it stands), and
// the index of the solve just done (the merge advanced it).
__global__ void repair_prep_kernel(const InstanceDesc* inst, InstanceDesc* rep)
{
    if (threadIdx.x == 0) {
        rep->cur = inst->cur;
        rep->vshift = 0;
        rep->solve_index = inst->solve_index - 1u;
    }
}

// The repaired controls (the rollout's single-precision record of them) replace v+ in place, and
// v_safe_0 becomes the returned command.
__global__ __launch_bounds__(256) void repair_finish_kernel(InstanceDesc* inst,
                                                            const InstanceDesc* rep)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < 2 * inst->T) {
        const double val = (double)rep->u[i];
        inst->v[inst->cur][i] = val;
        if (i < 2) inst->stats[5 + i] = val;
    }
}

// Merge for the stand-alone K-reduction (explicit buffers, no instance state).
__global__ __launch_bounds__(256) void merge_plain_kernel(int T, int G, double lambda,
                                                          const double* partial,
                                                          const double* v_in, double* v_out,
                                                          double* stats)
{
    const int col = (int)(blockIdx.x * 4u + (threadIdx.x >> 6));
    if (col >= 2 * T) return;
    double m, Z, W2, nf, N;
    merge_entry(partial, G, T, col, lambda, m, Z, W2, nf, N);
    if ((threadIdx.x & 63u) == 0) {
        const bool ok = nf > 0.0 && Z > 0.0;
        const double vo = ok ? v_in[col] + N / Z : v_in[col];
        v_out[col] = vo;
        write_stats(stats, col, vo, ok, m, Z, W2, nf);
    }
}

// ----------------------------------------------------------------------------------------------
// stand-alone kernels for staged checks
// ----------------------------------------------------------------------------------------------
// scoring from given beliefs: one wave per sample, records in chunks of 64 lanes
__global__ __launch_bounds__(256) void score_kernel(int K, int T, ScoreF64 sc, const double* mom,
                                                    const float* u, const double* v, double* S)
{
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int k = blockIdx.x * 4 + w;
    if (k >= K) return;
    const double* mk = mom + (size_t)k * (T + 1) * 9;
    const float2* uk = reinterpret_cast<const float2*>(u) + (size_t)k * T;
    double part = 0.0, h_carry = 0.0;
    for (int base = 0; base <= T; base += 64) {
        const int count = min(64, T + 1 - base);
        const int rec = base + min(lane, count - 1);
        part += score_chunk(sc, mk + (size_t)rec * 9, base + lane, count, lane, 64, T, uk, v, 0,
                            h_carry);
    }
    part = group_sum(part, 64);
    if (lane == 0) S[k] = part;
}

// K-reduction partials from given costs and controls (kPartialSlice samples per block)
__global__ __launch_bounds__(256) void partial_kernel(int K, int T, double lambda, const double* S,
                                                      const float* u, const double* v,
                                                      double* partial)
{
    extern __shared__ double psm[];
    double* S_sh = psm;
    double* w_sh = psm + kPartialSlice;
    float2* u_sh = reinterpret_cast<float2*>(psm + 2 * kPartialSlice);
    const int k0 = blockIdx.x * kPartialSlice;
    const int n = min(kPartialSlice, K - k0);
    if (threadIdx.x < n) S_sh[threadIdx.x] = S[k0 + threadIdx.x];
    const float2* uu = reinterpret_cast<const float2*>(u) + (size_t)k0 * T;
    for (int i = threadIdx.x; i < n * T; i += 256) u_sh[i] = uu[i];
    __syncthreads();
    block_partial(T, n, S_sh, w_sh, u_sh, v, 0, lambda, partial + (size_t)blockIdx.x * (2 * T + 4));
}

__global__ void philox_kernel(uint32_t k0, uint32_t k1, const uint32_t* ctr, uint32_t* out,
                              int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c0 = ctr[4 * i], c1 = ctr[4 * i + 1], c2 = ctr[4 * i + 2], c3 = ctr[4 * i + 3];
    philox10(c0, c1, c2, c3, k0, k1);
    out[4 * i] = c0;
    out[4 * i + 1] = c1;
    out[4 * i + 2] = c2;
    out[4 * i + 3] = c3;
}

__global__ void normals_kernel(uint32_t k0, uint32_t k1, const uint32_t* ctr, float* z, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c0 = ctr[4 * i], c1 = ctr[4 * i + 1], c2 = ctr[4 * i + 2], c3 = ctr[4 * i + 3];
    philox10(c0, c1, c2, c3, k0, k1);
    float z0, z1, z2, z3;
    bm_pair(c0, c1, z0, z1);
    bm_pair(c2, c3, z2, z3);
    z[4 * i] = z0;
    z[4 * i + 1] = z1;
    z[4 * i + 2] = z2;
    z[4 * i + 3] = z3;
}

__global__ void model_step_kernel(CarF32 car, const float* x, const float* u, float* xn, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* xi = x + 6 * i;
    const StepF32 st = make_step(car, u[2 * i], u[2 * i + 1]);
    float Xs = xi[0], Xc = 0.0f, Ys = xi[1], Yc = 0.0f, Ps = xi[2], Pc = 0.0f;
    float vx = xi[3], vy = xi[4], vr = xi[5];
    float dX1, dY1, dvx1, dvy1, dr1;
    car_field_f32(car, st, Ps * kInv2Pi, vx, vy, vr, dX1, dY1, dvx1, dvy1, dr1);
    const float pm = fmaf(car.half_dt, vr, Ps);
    const float vxm = fmaf(car.half_dt, dvx1, vx);
    const float vym = fmaf(car.half_dt, dvy1, vy);
    const float vrm = fmaf(car.half_dt, dr1, vr);
    float dX2, dY2, dvx2, dvy2, dr2;
    car_field_f32(car, st, pm * kInv2Pi, vxm, vym, vrm, dX2, dY2, dvx2, dvy2, dr2);
    kahan_add(Xs, Xc, car.dt * dX2);
    kahan_add(Ys, Yc, car.dt * dY2);
    kahan_add(Ps, Pc, car.dt * vrm);
    float* o = xn + 6 * i;
    o[0] = Xs - Xc;
    o[1] = Ys - Yc;
    o[2] = Ps - Pc;
    o[3] = fmaf(car.dt, dvx2, vx);
    o[4] = fmaf(car.dt, dvy2, vy);
    o[5] = fmaf(car.dt, dr2, vr);
}

__global__ void sdf_kernel(EllipseF64 E, const double* pts, double* out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double sd, nx, ny;
    ellipse_sdf(E, pts[2 * i], pts[2 * i + 1], &sd, &nx, &ny);
    out[3 * i] = sd;
    out[3 * i + 1] = nx;
    out[3 * i + 2] = ny;
}

__global__ void repair_kernel(ScoreF64 sc, const double* mom, const double* u_in, double* u_out,
                              int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* bel = mom + 9 * i;
    double us0 = u_in[2 * i], us1 = u_in[2 * i + 1];
    if (sc.shield_iters > 0) {
        const BeliefEval be = eval_belief(sc, bel);
        const double fd = sc.shield_fd;
        for (int it = 0; it < sc.shield_iters; ++it) {
            const double r0 = repair_residual(sc, bel, be, be.h, us0, us1);
            if (!(r0 > 0.0)) break;
            const double g0 = (repair_residual(sc, bel, be, be.h, us0 + fd, us1) -
                               repair_residual(sc, bel, be, be.h, us0 - fd, us1)) / (2.0 * fd);
            const double g1 = (repair_residual(sc, bel, be, be.h, us0, us1 + fd) -
                               repair_residual(sc, bel, be, be.h, us0, us1 - fd)) / (2.0 * fd);
            const double den = g0 * g0 + g1 * g1 + sc.shield_gmin * sc.shield_gmin;
            us0 = clampd(us0 - r0 * g0 / den, -sc.steer_max, sc.steer_max);
            us1 = clampd(us1 - r0 * g1 / den, -sc.accel_max, sc.accel_max);
        }
    }
    u_out[2 * i] = us0;
    u_out[2 * i + 1] = us1;
}

template <int P>
hipError_t launch_solve_p(const InstanceDesc* inst, const BlockDesc* blocks, int nblocks,
                          bool shield, bool split, bool resample, bool con, size_t lds,
                          const double* x0_base, const double* Sigma0_base, int extra_shift,
                          hipStream_t stream)
{
    const dim3 g(nblocks), b256(256), b512(512);
    if (con && (shield || resample))
        hipLaunchKernelGGL((solve_kernel<P, true, false, true, true>), g, b256, lds, stream, inst,
                           blocks, x0_base, Sigma0_base, extra_shift);
    else if (con && split)
        hipLaunchKernelGGL((solve_kernel<P, false, true, false, true>), g, b512, lds, stream, inst,
                           blocks, x0_base, Sigma0_base, extra_shift);
    else if (con)
        hipLaunchKernelGGL((solve_kernel<P, false, false, false, true>), g, b256, lds, stream, inst,
                           blocks, x0_base, Sigma0_base, extra_shift);
    else if (shield && resample)
        hipLaunchKernelGGL((solve_kernel<P, true, false, true>), g, b256, lds, stream, inst,
                           blocks, x0_base, Sigma0_base, extra_shift);
    else if (shield)
        hipLaunchKernelGGL((solve_kernel<P, true, false, false>), g, b256, lds, stream, inst,
                           blocks, x0_base, Sigma0_base, extra_shift);
    else if (resample)
        hipLaunchKernelGGL((solve_kernel<P, false, false, true>), g, b256, lds, stream, inst,
                           blocks, x0_base, Sigma0_base, extra_shift);
    else if (split)
        hipLaunchKernelGGL((solve_kernel<P, false, true, false>), g, b512, lds, stream, inst,
                           blocks, x0_base, Sigma0_base, extra_shift);
    else
        hipLaunchKernelGGL((solve_kernel<P, false, false, false>), g, b256, lds, stream, inst,
                           blocks, x0_base, Sigma0_base, extra_shift);
    return hipGetLastError();
}

unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// particles per lane: the smallest of 1, 2, 4, 8 covering M with the given lanes
static int ppl_for(int M, int lanes)
{
    const int need = (M + lanes - 1) / lanes;
    int p = 1;
    while (p < need) p <<= 1;
    return p;
}

size_t solve_lds_bytes(int lanes, int T, int ppl, bool split)
{
    const int groups = 256 / lanes;
    return (size_t)2 * groups * sizeof(double) + (size_t)groups * T * sizeof(float2) +
           (split ? (size_t)2 * ppl * 3 * 256 * sizeof(float) : 0);
}

bool split_pays(int nblocks, int lanes, int T, int ppl)
{
    // fewer than two waves per SIMD (256 CUs x 4 SIMDs, four waves per block), and room for the
    // noise ring
    return (int64_t)nblocks * 4 < 2 * 1024 && solve_lds_bytes(lanes, T, ppl, true) <= kMaxLds;
}

LaunchShape choose_shape(int K, int M, int T, int requested_lanes, int requested_ppl,
                         int requested_split, bool shield)
{
    LaunchShape s;
    const bool lanes_ok = requested_lanes == 8 || requested_lanes == 16 || requested_lanes == 32 ||
                          requested_lanes == 64;
    if (requested_ppl == 1 || requested_ppl == 2 || requested_ppl == 4 || requested_ppl == 8) {
        // lanes follow from the particles per lane: the smallest power of two >= 8 with L P >= M
        // (the shield's difference points need five lanes per group)
        int lanes = 8;
        while (lanes < 64 && lanes * requested_ppl < M) lanes <<= 1;
        s.lanes = lanes;
    } else if (lanes_ok) {
        s.lanes = requested_lanes;
    } else if (shield) {
        // default with the repair: eight particles per lane, so that a wave holds as many samples
        // as possible (the repair runs in five lanes of every group while the wave executes it
        // once for all its groups: its cost is per wave, not per sample)
        int lanes = 8;
        while (lanes < 64 && lanes * 8 < M) lanes <<= 1;
        s.lanes = lanes;
    } else {
        // default: about four particles per lane, 16..64 lanes per sample
        int lanes = 16;
        while (lanes < 64 && lanes * 4 < M) lanes <<= 1;
        s.lanes = lanes;
    }
    s.ppl = ppl_for(M, s.lanes);
    while ((s.ppl > 8 || solve_lds_bytes(s.lanes, T, s.ppl, false) > kMaxLds) && s.lanes < 64) {
        s.lanes <<= 1;
        s.ppl = ppl_for(M, s.lanes);
    }
    const bool fits = solve_lds_bytes(s.lanes, T, s.ppl, true) <= kMaxLds;
    s.split = requested_split > 0 ? fits
              : requested_split == 0 ? false
                                     : split_pays(solve_blocks(K, s.lanes), s.lanes, T, s.ppl);
    return s;
}

int solve_blocks(int K, int lanes)
{
    const int groups = 256 / lanes;
    return (K + groups - 1) / groups;
}

hipError_t launch_solve(const InstanceDesc* inst, const BlockDesc* blocks, int nblocks, int ppl,
                        bool shield, bool split, bool resample, bool con, size_t lds,
                        const double* x0_base, const double* Sigma0_base, int extra_shift,
                        hipStream_t stream)
{
    if (nblocks <= 0) return hipSuccess;
    split = split && !shield && !resample;
    switch (ppl) {
    case 1:
        return launch_solve_p<1>(inst, blocks, nblocks, shield, split, resample, con,
                                    lds, x0_base, Sigma0_base, extra_shift, stream);
    case 2:
        return launch_solve_p<2>(inst, blocks, nblocks, shield, split, resample, con,
                                    lds, x0_base, Sigma0_base, extra_shift, stream);
    case 4:
        return launch_solve_p<4>(inst, blocks, nblocks, shield, split, resample, con,
                                    lds, x0_base, Sigma0_base, extra_shift, stream);
    case 8:
        return launch_solve_p<8>(inst, blocks, nblocks, shield, split, resample, con,
                                    lds, x0_base, Sigma0_base, extra_shift, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_merge(const InstanceDesc* inst, const MergeDesc* cols, int ncols,
                        int extra_shift, hipStream_t stream)
{
    if (ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL(merge_kernel, dim3(blocks_for(ncols, 4)), dim3(256), 0, stream,
                       const_cast<InstanceDesc*>(inst), cols, ncols, extra_shift);
    return hipGetLastError();
}

hipError_t launch_local_repair(InstanceDesc* inst, InstanceDesc* rep, const BlockDesc* rep_block,
                               int T, int ppl, bool resample, bool con, size_t lds,
                               const double* x0_base, const double* Sigma0_base,
                               hipStream_t stream)
{
    hipLaunchKernelGGL(repair_prep_kernel, dim3(1), dim3(64), 0, stream, inst, rep);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_solve(rep, rep_block, 1, ppl, true, false, resample, con, lds, x0_base,
                     Sigma0_base, 0, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(repair_finish_kernel, dim3(blocks_for(2 * T, 256)), dim3(256), 0, stream,
                       inst, rep);
    return hipGetLastError();
}

hipError_t launch_merge_plain(int T, int G, double lambda, const double* partial,
                              const double* v_in, double* v_out, double* stats,
                              hipStream_t stream)
{
    hipLaunchKernelGGL(merge_plain_kernel, dim3(blocks_for(2 * T, 4)), dim3(256), 0, stream, T,
                       G, lambda, partial, v_in, v_out, stats);
    return hipGetLastError();
}

hipError_t launch_score(int K, int T, const ScoreF64& sc, const double* mom, const float* u,
                        const double* v, double* S, hipStream_t stream)
{
    hipLaunchKernelGGL(score_kernel, dim3(blocks_for(K, 4)), dim3(256), 0, stream, K, T, sc, mom,
                       u, v, S);
    return hipGetLastError();
}

int partial_blocks(int K) { return (K + kPartialSlice - 1) / kPartialSlice; }

hipError_t launch_partials(int K, int T, double lambda, const double* S, const float* u,
                           const double* v, double* partial, hipStream_t stream)
{
    const size_t lds = (size_t)2 * kPartialSlice * sizeof(double) +
                       (size_t)kPartialSlice * T * sizeof(float2);
    hipLaunchKernelGGL(partial_kernel, dim3(partial_blocks(K)), dim3(256), lds, stream, K, T,
                       lambda, S, u, v, partial);
    return hipGetLastError();
}

hipError_t launch_philox(uint32_t key0, uint32_t key1, const uint32_t* ctr, uint32_t* out,
                         int64_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(philox_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, stream, key0, key1,
                       ctr, out, n);
    return hipGetLastError();
}

hipError_t launch_normals(uint32_t key0, uint32_t key1, const uint32_t* ctr, float* z, int64_t n,
                          hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(normals_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, stream, key0, key1,
                       ctr, z, n);
    return hipGetLastError();
}

hipError_t launch_model_step(const CarF32& car, const float* x, const float* u, float* xn,
                             int64_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(model_step_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, stream, car, x,
                       u, xn, n);
    return hipGetLastError();
}

hipError_t launch_sdf(double a, double b, const double* pts, double* out, int64_t n,
                      hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(sdf_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, stream,
                       make_ellipse(a, b), pts, out, n);
    return hipGetLastError();
}

hipError_t launch_repair(const ScoreF64& sc, const double* mom, const double* u_in, double* u_out,
                         int64_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(repair_kernel, dim3(blocks_for(n, 64)), dim3(64), 0, stream, sc, mom, u_in,
                       u_out, n);
    return hipGetLastError();
}

}  // namespace bss
