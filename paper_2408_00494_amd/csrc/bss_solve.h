// bss_solve.h -- the solve kernel of one BSS-MPPI solve (gfx950), compiled once per
// particles-per-lane count (bss_solve_p{1,2,4,8}.hip) so that the variants build in parallel.
//
// L lanes per control sample k (256/L samples per 256-thread block), P particles per lane in
// registers.  Draws eps_{k,t} (Philox tag 0) lane-parallel over t, optionally shield-repairs
// u_{k,t} per step, propagates the M particles with the single-precision midpoint rule plus the
// disturbance (tag 1), reduces the particle mean and position covariance across the L lanes in
// double precision every step (the belief record of each step goes to a [K][T+1][9] buffer),
// then scores the belief trajectory L records at a time (one per lane: signed distance, sigma_y,
// barrier h, running cost, control cost, C_safe), and folds the block's samples into a
// log-sum-exp partial (weights relative to the block's own minimum cost).  Scoring after the
// particle loop keeps its double-precision temporaries out of the loop's register budget.
#pragma once

#include "bss_wave.h"

namespace bss {

namespace {

// ----------------------------------------------------------------------------------------------
// solve: rollout + scoring + block partial of the K-reduction
// ----------------------------------------------------------------------------------------------
// Up to four particles per lane the loop fits 128 registers, which keeps four waves per SIMD;
// eight particles fit the budget of three, the shield's double-precision repair that of two.

// Disturbance normals of step t for the P particles of one lane, written to slot t & 1 of the
// ring [2][P][RW][256] (lane-contiguous, so the stores and the loads are conflict-free); with
// RW = 9 (the re-sampling loop) also the six standard normals of each particle's re-sampling draw
// at step t > 0 (counters (t, m, k, tag 4 or 5): the draw of resample_particles).
template <int P, int L, int RW>
__device__ __forceinline__ void produce_noise(float* ring, int t, int q, int j,
                                              const PhiloxParticle* pb, uint32_t c3w, uint32_t lk,
                                              uint32_t key0, uint32_t key1, bool draws = false,
                                              uint32_t s = 0u, int k = 0)
{
    const PhiloxStep ps = philox_step((uint32_t)t, c3w, lk, key0, key1);
    float* dst = ring + (t & 1) * (P * RW * 256) + q;
    NoiseDealer<P> deal{ps, pb, key0, key1, j, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int p = 0; p < P; ++p) {
        float w0, w1, w2;
        deal.next(p, w0, w1, w2);
        dst[(p * RW + 0) * 256] = w0;
        dst[(p * RW + 1) * 256] = w1;
        dst[(p * RW + 2) * 256] = w2;
    }
    if constexpr (RW == 9) {
        if (draws && t > 0) {
            const uint64_t pkr = (uint64_t)kPhiloxM1 * (uint32_t)k;
            const uint32_t hkr = (uint32_t)(pkr >> 32), lkr = (uint32_t)pkr;
            const PhiloxStep psr0 =
                philox_step((uint32_t)t, rng_word3(kTagResample0, s), lkr, key0, key1);
            const PhiloxStep psr1 =
                philox_step((uint32_t)t, rng_word3(kTagResample1, s), lkr, key0, key1);
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const uint32_t m = (uint32_t)particle_of<P, L>(j, p);
                const PhiloxParticle pm = philox_particle(m, hkr, key0, key1);
#pragma unroll
                for (int blk = 0; blk < 2; ++blk) {
                    uint32_t c0, c1, c2, c3;
                    philox10_tail(blk == 0 ? psr0 : psr1, pm, key0, key1, c0, c1, c2, c3);
                    float z0, z1;
                    bm_pair(c0, c1, z0, z1);
                    dst[(p * RW + 3 + 3 * blk + 0) * 256] = z0;
                    dst[(p * RW + 3 + 3 * blk + 1) * 256] = z1;
                    dst[(p * RW + 3 + 3 * blk + 2) * 256] = bm_cos(c2, c3);
                }
            }
        }
    }
}

// ---- moment exchange: per-lane partial moment sums totalled in LDS ----
// Pairwise sum of row[0..L): adjacent pairs, then pairs of pairs, and so on (one fixed order, so
// every variant that totals the same entries gets the same bits).
template <int L>
__device__ __forceinline__ double tree_sum(const double* row)
{
    if constexpr (L > 16) {
        return tree_sum<L / 2>(row) + tree_sum<L / 2>(row + L / 2);
    } else {
        double a[L];
#pragma unroll
        for (int i = 0; i < L; ++i) a[i] = row[i];
#pragma unroll
        for (int w = 1; w < L; w <<= 1)
#pragma unroll
            for (int i = 0; i < L; i += 2 * w) a[i] += a[i + w];
        return a[0];
    }
}

// Entry r of a belief record (mean X, Y, psi, vx, vy, r; covariance XX, XY, YY) from the group
// totals: tot = row r's total, s0 / s1 = the totals of the shifted positions (rows 0 and 1),
// ref = the reference position's coordinate (rows 0 and 1, else 0), x0r = the estimate's entry
// (rows 0 to 2, else 0).
__device__ __forceinline__ double belief_entry(int r, double tot, double s0, double s1, double ref,
                                               double x0r, double invM, double invM1)
{
    // no contraction: every variant rounds these operations the same way
#pragma clang fp contract(off)
    if (r < 3) return x0r + (ref + tot * invM);
    if (r < 6) return tot * invM;
    const double a = r == 8 ? s1 : s0;
    const double b = (r == 6 ? s0 : s1) * invM;
    return fma(-a, b, tot) * invM1;
}

// Totals of rows [0, nr) of a group's region (lane i of the group totals rows i, i + L, ...),
// stored after each row's L entries.  The entries must be visible to the calling wave.
template <int L>
__device__ __forceinline__ void total_rows(double* reg, int j, int nr)
{
#pragma unroll
    for (int r0 = 0; r0 < moment_rows(true); r0 += L) {
        const int r = r0 + j;
        if (r < nr) reg[r * (L + 1) + L] = tree_sum<L>(reg + r * (L + 1));
    }
    wave_lds_sync();
}

// Writes the nine entries of a belief record from a totalled region, entry r by lane r of the
// group (and r + 8 by lane r when L = 8).
template <int L>
__device__ __forceinline__ void record_from_totals(const double* reg, int j, double refX,
                                                   double refY, const double (&x0)[6],
                                                   double invM, double invM1, double* rec)
{
    constexpr int ROW = L + 1;
    const double s0 = reg[L], s1 = reg[ROW + L];
#pragma unroll
    for (int r0 = 0; r0 < 9; r0 += L) {
        const int r = r0 + j;
        if (r < 9) {
            const double ref = r == 0 ? refX : (r == 1 ? refY : 0.0);
            const double x0r = r == 0 ? x0[0] : (r == 1 ? x0[1] : (r == 2 ? x0[2] : 0.0));
            rec[r] = belief_entry(r, reg[r * ROW + L], s0, s1, ref, x0r, invM, invM1);
        }
    }
}

// Unbiased variance of a half-space constraint's projection a^T x over the particles (eq. 11 with
// eta_i = a_i) from a totalled region: the sum of the projections follows from the moment totals
// (rows 0 to 5, positions shifted by the reference, velocities about the estimate's), s2 is the
// total of the squared projections.  Sigma points add a^T Q a of the disturbance covariance,
// scaled like Q by the points' mean of (1 + kappa |vx|)^2.
__device__ __forceinline__ double con_variance(const double* a, const double* reg, int L,
                                               double s2, const double (&x0)[6], int M,
                                               double invM, double invM1, bool sigma, double qbar,
                                               float sw0, float sw1, float sw2)
{
#pragma clang fp contract(off)
    const int ROW = L + 1;
    const double s1 =
        fma(a[0], reg[L],
            fma(a[1], reg[ROW + L],
                fma(a[2], reg[2 * ROW + L],
                    fma(a[3], fma(-(double)M, x0[3], reg[3 * ROW + L]),
                        fma(a[4], fma(-(double)M, x0[4], reg[4 * ROW + L]),
                            a[5] * fma(-(double)M, x0[5], reg[5 * ROW + L]))))));
    double var = (s2 - s1 * (s1 * invM)) * invM1;
    if (sigma) {
        const double q0 = a[3] * (double)sw0, q1 = a[4] * (double)sw1, q2 = a[5] * (double)sw2;
        var = fma(qbar, fma(q0, q0, fma(q1, q1, q2 * q2)), var);
    }
    return var;
}

// Split loop: whether the noise waves total step t's moment sums (the integrating waves total the
// other steps' themselves, in the wave).  Chosen by measurement so that neither kind of wave waits
// long at the step barrier: every other step, and every step in the re-sampling variant (whose
// integrating waves also re-sample).
template <bool SPLIT, bool RESAMPLE>
__device__ __forceinline__ bool hand_over(int t)
{
    if constexpr (!SPLIT) return false;
    else if constexpr (RESAMPLE) return true;
    else return (t & 1) != 0;
}

// LDS of the re-sampling sums, one array for every lane count of a kernel (the largest need is 8
// lanes': group_sums_lds of 14 values).
constexpr int kResampleLdsDoubles = group_sums_lds_doubles<14, 8>();
static_assert(kResampleLdsDoubles * sizeof(double) == kResampleStaticLds, "re-sampling LDS size");
static_assert(group_sums_lds_doubles<14, 16>() <= kResampleLdsDoubles &&
                  group_sums_lds_doubles<14, 32>() <= kResampleLdsDoubles,
              "re-sampling LDS");

__device__ __forceinline__ double* resample_lds()
{
    __shared__ double buf[kResampleLdsDoubles];
    return buf;
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
// xi_src (split loop): the draws' normals of this lane's particles at step t in the noise ring
// (normal a of particle p at xi_src[(9 p + 3 + a) 256]), produced by the noise waves; nullptr:
// drawn here.
template <int P, int L>
__device__ __forceinline__ void resample_particles(int t, int j, int k, int M, uint32_t s,
                                                   uint32_t key0, uint32_t key1, int mode,
                                                   double qbar, const float* sw, float* Xs,
                                                   float* Xc, float* Ys, float* Yc, float* Ps,
                                                   float* Pc, float* vx, float* vy, float* vr,
                                                   const float* xi_src = nullptr)
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
        if (particle_of<P, L>(j, p) < M) {
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
    // the 27 sums over the group's lanes: through LDS (two passes of 14 and 13 values) for up to
    // 32 lanes, where DPP would take three moves and an add per sum and stage; across a whole
    // wave by DPP and the swap instructions
    if constexpr (L <= 32) {
        double* lds = resample_lds();
        double lo[14], hi[13];
#pragma unroll
        for (int a = 0; a < 6; ++a) lo[a] = sd[a];
        int n = 6;
#pragma unroll
        for (int a = 0; a < 6; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b) {
                if (n < 14) lo[n] = sq[a][b];
                else hi[n - 14] = sq[a][b];
                ++n;
            }
        group_sums_lds<14, L, 14>(lo, lds);
        group_sums_lds<13, L, 14>(hi, lds);
#pragma unroll
        for (int a = 0; a < 6; ++a) sd[a] = lo[a];
        n = 6;
#pragma unroll
        for (int a = 0; a < 6; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b) {
                sq[a][b] = n < 14 ? lo[n] : hi[n - 14];
                ++n;
            }
    } else {
#pragma unroll
        for (int a = 0; a < 6; ++a) sd[a] = group_sum(sd[a], L);
#pragma unroll
        for (int a = 0; a < 6; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b) sq[a][b] = group_sum(sq[a][b], L);
    }
    double mean[6], cov[6][6];
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        mean[a] = ref[a] + sd[a] * invM;
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const double c = (sq[a][b] - sd[a] * (sd[b] * invM)) * invM1;
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
    // the draws' counters (t, m, k, tag 4 or 5) share their first two rounds as the disturbance's
    // do: per step two parts common to the sample, per particle one
    const uint64_t pk = (uint64_t)kPhiloxM1 * (uint32_t)k;
    const uint32_t hk = (uint32_t)(pk >> 32), lk = (uint32_t)pk;
    PhiloxStep psr[2];
    if (mode != 2 && !xi_src) {
        psr[0] = philox_step((uint32_t)t, rng_word3(kTagResample0, s), lk, key0, key1);
        psr[1] = philox_step((uint32_t)t, rng_word3(kTagResample1, s), lk, key0, key1);
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint32_t m = (uint32_t)particle_of<P, L>(j, p);
        double xi[6];
        if (mode == 2) {
            // selects instead of a runtime index keep xi in registers
            const double r = m < 6u ? 2.449489742783178 : -2.449489742783178;
            const uint32_t e = m % 6u;
#pragma unroll
            for (int a = 0; a < 6; ++a) xi[a] = (m < 12u && e == (uint32_t)a) ? r : 0.0;
        } else if (xi_src) {
#pragma unroll
            for (int a = 0; a < 6; ++a) xi[a] = xi_src[(p * 9 + 3 + a) * 256];
        } else {
            const PhiloxParticle pm = philox_particle(m, hk, key0, key1);
#pragma unroll
            for (int blk = 0; blk < 2; ++blk) {
                uint32_t c0, c1, c2, c3;
                philox10_tail(psr[blk], pm, key0, key1, c0, c1, c2, c3);
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

// One solve block with L lanes per sample (L is a compile-time constant so that the loops over a
// group's lanes and the sample sums are straight-line code).
//
// SPLIT (512 threads): threads 256..511 generate the disturbance normals of step t + 1 while
// threads 0..255 integrate step t, through a two-slot LDS ring and one barrier per step; they
// also total the moment sums of the steps handed over to them (hand_over) and evaluate records in
// the scoring phase.  This puts two waves on every SIMD when a launch has too few samples to fill
// the chip otherwise (a lone wave issues at about half the SIMD's rate); the arithmetic and its
// order are unchanged, so the results are bitwise the same as without the split.
template <int P, bool SHIELD, int L, bool SPLIT, bool RESAMPLE, bool CON>
__device__ __forceinline__ void solve_block(const InstanceDesc& d, const BlockDesc bd,
                                            const double* __restrict__ x0_base,
                                            const double* __restrict__ Sigma0_base,
                                            int extra_shift)
{
    static_assert(!(SPLIT && SHIELD), "the shielded loop is not split");
    static_assert(!(SPLIT && RESAMPLE && CON), "the generic loop is not split");
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
    // SPLIT: [2][P][RW][256], RW = 3 disturbance normals per particle, 9 with the re-sampling
    // draw's six
    constexpr int RW = RESAMPLE ? 9 : 3;
    float* ring = reinterpret_cast<float*>(u_sh + groups * T);
    // moment exchange: [slots][groups][GR] doubles, two slots with the split (step t's sums are
    // totalled by the noise waves while step t + 1 is integrated), one without
    constexpr int NR = moment_rows(CON);
    constexpr int GR = moment_region_doubles(L, CON);
    double* mscr = reinterpret_cast<double*>(ring + (SPLIT ? 2 * P * RW * 256 : 0));
    // on-chip belief records (rec_lds): [groups][T+1][9], then [groups][T+1][n_con]
    double* rec_sh = mscr + (SPLIT ? 2 : 1) * groups * GR;
    const int q = SPLIT ? (int)(threadIdx.x & 255u) : (int)threadIdx.x;
    const bool producer = SPLIT && threadIdx.x >= 256u;
    const int g = q >> log2L;
    const int j = q & (L - 1);
    const int k = bd.k0 + g;
    const bool active = k < d.K;
    float2* us = u_sh + g * T;
    // the records of this sample: in HBM (mom, an output) or in the block's LDS (generic pointers
    // either way; the scoring phase reads them back from the same block)
    double* mom_k = d.rec_lds ? rec_sh + (size_t)g * (T + 1) * 9
                              : d.mom + (size_t)(active ? k : 0) * (T + 1) * 9;
    const uint32_t s = d.solve_index;
    const uint32_t key0 = d.key0, key1 = d.key1;
    const double* x0p = x0_base + 6 * d.x0_index;
    const double* S0p = Sigma0_base ? Sigma0_base + 36 * d.x0_index : nullptr;
    // half-space constraints on the whole state (compiled into the CON variants only): their
    // variances a_i^T Sigma a_i per record
    const int ncon = CON ? d.sc.n_con : 0;
    double* cvar_k =
        ncon == 0 ? nullptr
        : d.rec_lds ? rec_sh + (size_t)groups * (T + 1) * 9 + (size_t)g * (T + 1) * ncon
                    : d.cvar + (size_t)(active ? k : 0) * (T + 1) * ncon;

    // ---- phase 1: control samples u_{k,t} = clip(v_t + eps_{k,t}), lane-parallel over t (with
    // the split by the integrating waves, while the noise waves draw step 0's normals) ----
    if (active && !producer) {
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
    constexpr int NB = noise_blocks<P>();
    if (SPLIT && producer && active) {
        PhiloxParticle pb0[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i)
            pb0[i] = philox_particle(noise_block_word<P, L>(j, i), hk, key0, key1);
        produce_noise<P, L, RW>(ring, 0, q, j, pb0, c3w, lk, key0, key1);
    }
    __syncthreads();

    if (SPLIT || active) {
        const bool consumer = !producer && active;
        double x0[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) x0[i] = x0p[i];
        const bool spread = S0p != nullptr;
        // half-space directions in registers, with a_i^T of the estimate's velocities folded into
        // one constant: a_i^T (x - xref) = a_i^T (X, Y, psi, vx, vy, r) - cb_i (the plain and
        // split constraint variants; the generic one has no registers to spare)
        constexpr bool HOIST = CON && !SHIELD && !RESAMPLE;
        double ca[HOIST ? kMaxCon : 1][6], cb[HOIST ? kMaxCon : 1];
        if constexpr (HOIST) {
#pragma unroll
            for (int c = 0; c < kMaxCon; ++c) {
#pragma unroll
                for (int e = 0; e < 6; ++e) ca[c][e] = c < ncon ? d.sc.con_a[6 * c + e] : 0.0;
                cb[c] = fma(ca[c][3], x0[3], fma(ca[c][4], x0[4], ca[c][5] * x0[5]));
            }
        }

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
                const int m = particle_of<P, L>(j, p);
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
        PhiloxParticle pb[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i)
            pb[i] = philox_particle(noise_block_word<P, L>(j, i), hk, key0, key1);
        const double invM = 1.0 / (double)M;
        const double invM1 =
            (RESAMPLE && d.belief == 2) ? invM : (M > 1 ? 1.0 / (double)(M - 1) : 0.0);
        const float swv[3] = {sw0, sw1, sw2};
        double qbar = 1.0;      // sigma points: previous points' mean of (1 + kappa |vx|)^2

        // Record rt from a group region holding the lanes' partial sums of step rt - 1 (and, for
        // the variants that repair or carry constraints, the belief and the constraint variances
        // of record rt in every lane of the group).  Run by the integrating waves right after
        // their sums, or with the split by the noise waves during the next step.
        auto finish_moments = [&](double* reg, int rt, double rX, double rY) {
            constexpr int ROW = L + 1;
            total_rows<L>(reg, j, 9 + ncon);
            if constexpr (!SHIELD) {
                // the belief feeds only the records: entry r by lane r, constraint c's variance
                // by lane 9 + c (lane 1 + c of the second pass when L = 8)
                record_from_totals<L>(reg, j, rX, rY, x0, invM, invM1, mom_k + (size_t)rt * 9);
                if constexpr (CON) {
#pragma unroll
                    for (int r0 = 0; r0 < NR; r0 += L) {
                        const int c = r0 + j - 9;
                        if (c >= 0 && c < ncon)
                            cvar_k[(size_t)rt * ncon + c] =
                                con_variance(d.sc.con_a + 6 * c, reg, L, reg[(9 + c) * ROW + L],
                                             x0, M, invM, invM1, d.belief == 2, qbar, sw0, sw1,
                                             sw2);
                    }
                }
            } else {
                // the repair of the next step needs the belief in every lane
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    bel[i] = belief_entry(i, reg[i * ROW + L], reg[L], reg[ROW + L],
                                          i == 0 ? rX : (i == 1 ? rY : 0.0), i < 3 ? x0[i] : 0.0,
                                          invM, invM1);
#pragma unroll
                for (int c = 0; c < kMaxCon; ++c)
                    if (c < ncon)
                        bcv[c] = con_variance(d.sc.con_a + 6 * c, reg, L,
                                              reg[(9 + c < NR ? 9 + c : 0) * ROW + L], x0, M,
                                              invM, invM1, d.belief == 2, qbar, sw0, sw1, sw2);
                // record rt, written by lane rt % L of the group (spreads the stores)
                if (j == (rt & (L - 1))) {
                    double* rec = mom_k + (size_t)rt * 9;
#pragma unroll
                    for (int i = 0; i < 9; ++i) rec[i] = bel[i];
#pragma unroll
                    for (int c = 0; c < kMaxCon; ++c)
                        if (c < ncon) cvar_k[(size_t)rt * ncon + c] = bcv[c];
                }
            }
            wave_lds_sync();   // the region is written again by the next step
        };

        // In split mode every thread runs every iteration and meets exactly one barrier per step,
        // outside all divergent branches (waves may hold both active and inactive samples).
        for (int t = 0; t < T; ++t) {
            if (SPLIT && producer) {
                if (active && t + 1 < T)
                    produce_noise<P, L, RW>(ring, t + 1, q, j, pb, c3w, lk, key0, key1,
                                            RESAMPLE && d.belief == 1, s, k);
                if (active && t > 0 && hand_over<SPLIT, RESAMPLE>(t - 1)) {
                    double* reg = mscr + (size_t)(((t - 1) & 1) * groups + g) * GR;
                    finish_moments(reg, t, reg[NR * (L + 1)], reg[NR * (L + 1) + 1]);
                }
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
                    resample_particles<P, L>(
                        t, j, k, M, s, key0, key1, d.belief, qbar, swv, Xs, Xc, Ys, Yc, Ps, Pc,
                        vx, vy, vr,
                        SPLIT ? ring + (t & 1) * (P * RW * 256) + q : nullptr);
                if (RESAMPLE && d.belief == 2) {
                    double qs = 0.0;
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        if (particle_of<P, L>(j, p) < M) {
                            const double f = 1.0 + (double)ksp * fabs((double)vx[p]);
                            qs = fma(f, f, qs);
                        }
                    }
                    qbar = group_sum(qs, L) * invM;
                }
                const StepF32 st = make_step(car, uu.x, uu.y);
                PhiloxStep ps{};
                if (!SPLIT) ps = philox_step((uint32_t)t, c3w, lk, key0, key1);
                NoiseDealer<P> deal{ps, pb, key0, key1, j, 0.0f, 0.0f, 0.0f};
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
                            const float* src = ring + (t & 1) * (P * RW * 256) + q;
                            w0[i] = src[(p * RW + 0) * 256];
                            w1[i] = src[(p * RW + 1) * 256];
                            w2[i] = src[(p * RW + 2) * 256];
                        } else {
                            deal.next(p, w0[i], w1[i], w2[i]);
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
                        if (particle_of<P, L>(j, p) < M) {
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
                            if constexpr (HOIST) {
                                const double Pd = (double)Ps[p] - (double)Pc[p];
#pragma unroll
                                for (int c = 0; c < kMaxCon; ++c) {
                                    if (c < ncon) {
                                        const double y = fma(
                                            ca[c][0], X,
                                            fma(ca[c][1], Y,
                                                fma(ca[c][2], Pd,
                                                    fma(ca[c][3], (double)vx[p],
                                                        fma(ca[c][4], (double)vy[p],
                                                            fma(ca[c][5], (double)vr[p],
                                                                -cb[c]))))));
                                        c2[c] = fma(y, y, c2[c]);
                                    }
                                }
                            } else {
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
                }
                // moment exchange: the lane's partial sums into its group's rows
                {
                    constexpr int ROW = L + 1;
                    double* reg = mscr + (size_t)((SPLIT ? (t & 1) * groups : 0) + g) * GR;
                    reg[0 * ROW + j] = sX;
                    reg[1 * ROW + j] = sY;
                    reg[2 * ROW + j] = sP;
                    reg[3 * ROW + j] = svx;
                    reg[4 * ROW + j] = svy;
                    reg[5 * ROW + j] = svr;
                    reg[6 * ROW + j] = sXX;
                    reg[7 * ROW + j] = sXY;
                    reg[8 * ROW + j] = sYY;
#pragma unroll
                    for (int c = 0; c < kMaxCon; ++c)
                        if (CON && c < ncon) reg[(9 + c < NR ? 9 + c : 0) * ROW + j] = c2[c];
                    if (hand_over<SPLIT, RESAMPLE>(t)) {
                        // totalled by the noise waves during the next step
                        if (j == 0) {
                            reg[NR * ROW] = refX;
                            reg[NR * ROW + 1] = refY;
                        }
                    } else {
                        wave_lds_sync();
                        finish_moments(reg, t + 1, refX, refY);
                    }
                }
            }
            if (SPLIT) __syncthreads();
        }
        // the noise waves total the last step's sums when it was handed over
        if (SPLIT && producer && active && T > 0 && hand_over<SPLIT, RESAMPLE>(T - 1)) {
            double* reg = mscr + (size_t)(((T - 1) & 1) * groups + g) * GR;
            finish_moments(reg, T, reg[NR * (L + 1)], reg[NR * (L + 1) + 1]);
        }
    }
    // ---- phase 3: score the belief trajectory ----
    // In windows of W records per sample (a multiple of L, as many as the ring and the exchange,
    // free now, hold): every thread of the block evaluates records of the window, cost q and
    // barrier value h into LDS; then lane j of each group adds up its records j, j + L, ... of the
    // window with C_safe on the transitions into them.  The same form in every variant (the same
    // arithmetic wherever a record is scored).
    __threadfence_block();
    __syncthreads();
    double S_part = 0.0, V_part = 0.0;
    {
        constexpr int NT = SPLIT ? 512 : 256;
        double* qh = reinterpret_cast<double*>(ring);   // [groups][W][q, h]
        const int free_doubles = (SPLIT ? P * RW * 256 : 0) + (SPLIT ? 2 : 1) * groups * GR;
        const int W = free_doubles / (2 * groups) / L * L;
        const int nact = min(groups, d.K - bd.k0);
        double h_before = 0.0;   // h of the record before the window (record 0 has no transition)
        for (int w0 = 0; w0 <= T; w0 += W) {
            const int wn = min(W, T + 1 - w0);
            for (int r = (int)threadIdx.x; r < nact * wn; r += NT) {
                const int gg = r / wn, tt = w0 + (r - gg * wn);
                const size_t kr = (size_t)(bd.k0 + gg) * (T + 1) + tt;
                const size_t lr = (size_t)gg * (T + 1) + tt;
                const double* recp = d.rec_lds ? rec_sh + lr * 9 : d.mom + kr * 9;
                const double* crec = ncon == 0 ? nullptr
                                     : d.rec_lds ? rec_sh + (size_t)groups * (T + 1) * 9 + lr * ncon
                                                 : d.cvar + kr * ncon;
                double h;
                const double q = record_cost(d.sc, recp, tt, T, u_sh + gg * T, v, vshift, crec, h);
                qh[2 * (gg * W + (tt - w0))] = q;
                qh[2 * (gg * W + (tt - w0)) + 1] = h;
            }
            __syncthreads();
            if (active && !producer) {
                const double* qg = qh + (size_t)g * W * 2;
                for (int base = 0; base < wn; base += L) {
                    const int i = base + j;
                    double part = 0.0;
                    if (i < wn) {
                        part = qg[2 * i];
                        if (w0 + i >= 1)
                            part += transition_cost(d.sc, qg[2 * i + 1],
                                                    i > 0 ? qg[2 * i - 1] : h_before, &V_part);
                    }
                    S_part += part;
                }
                h_before = qg[2 * (wn - 1) + 1];
            }
            __syncthreads();   // the next window overwrites the records' (q, h)
        }
    }
    const double S_k = group_sum(S_part, L);
    const double V_k = group_sum(V_part, L);
    __shared__ double viol_sh[32];           // DCBF violations per group (at most 32 groups)
    if (j == 0 && !producer) {
        S_sh[g] = active ? S_k : INFINITY;
        viol_sh[g] = active ? V_k : 0.0;
        if (active) d.S[k] = S_k;
    }
    __syncthreads();
    const int n = min(groups, d.K - bd.k0);
    double nviol = 0.0;
    for (int i = 0; i < n; ++i) nviol += viol_sh[i];
    block_partial(T, n, S_sh, w_sh, u_sh, v, vshift, d.sc.lambda, nviol,
                  d.partial + (size_t)(bd.k0 >> (8 - log2L)) * partial_stride(T));
}

// One block of instance d with its lane count L taken from the descriptor (uniform over a block,
// so the dispatch is a block-uniform branch).
template <int P, bool SHIELD, bool SPLIT, bool RESAMPLE, bool CON>
__device__ __forceinline__ void solve_lanes_block(const InstanceDesc& d, const BlockDesc bd,
                                                  const double* __restrict__ x0_base,
                                                  const double* __restrict__ Sigma0_base,
                                                  int extra_shift)
{
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

// One block of the solve grid: the block looks up its instance and first sample.  P = 0 takes
// the particles per lane from the instance as well (a batch whose members run different P in one
// launch); the kernel's registers are then those of its largest P.
template <int P, bool SHIELD, bool SPLIT, bool RESAMPLE, bool CON>
__device__ __forceinline__ void solve_any_block(const InstanceDesc* __restrict__ insts,
                                                const BlockDesc bd,
                                                const double* __restrict__ x0_base,
                                                const double* __restrict__ Sigma0_base,
                                                int extra_shift)
{
    const InstanceDesc& d = insts[bd.inst];
    if constexpr (P == 0) {
        switch (d.ppl) {
        case 1:
            solve_lanes_block<1, SHIELD, SPLIT, RESAMPLE, CON>(d, bd, x0_base, Sigma0_base,
                                                               extra_shift);
            break;
        case 2:
            solve_lanes_block<2, SHIELD, SPLIT, RESAMPLE, CON>(d, bd, x0_base, Sigma0_base,
                                                               extra_shift);
            break;
        case 4:
            solve_lanes_block<4, SHIELD, SPLIT, RESAMPLE, CON>(d, bd, x0_base, Sigma0_base,
                                                               extra_shift);
            break;
        default:
            solve_lanes_block<8, SHIELD, SPLIT, RESAMPLE, CON>(d, bd, x0_base, Sigma0_base,
                                                               extra_shift);
            break;
        }
    } else {
        solve_lanes_block<P, SHIELD, SPLIT, RESAMPLE, CON>(d, bd, x0_base, Sigma0_base,
                                                           extra_shift);
    }
}

// The block body as a call of its own, for the persistent loop: inlined into the loop, the body
// takes more registers than the one-shot kernel and spills; out of line it keeps its own
// allocation, at the price of saving and restoring the callee-saved registers once per entry.
template <int P, bool SHIELD, bool SPLIT, bool RESAMPLE, bool CON>
__device__ __attribute__((noinline)) void solve_any_block_call(
    const InstanceDesc* __restrict__ insts, const BlockDesc bd,
    const double* __restrict__ x0_base, const double* __restrict__ Sigma0_base, int extra_shift)
{
    solve_any_block<P, SHIELD, SPLIT, RESAMPLE, CON>(insts, bd, x0_base, Sigma0_base,
                                                     extra_shift);
}

// Solve grid: every block looks up its instance and first sample; the lane count is uniform over
// a block, so the dispatch is a block-uniform branch.  PERSIST: the grid is persistent, each
// resident block takes the next entry of the block table from a work-queue counter (zeroed before
// the launch) until the table is exhausted, so a batch's blocks (ordered longest first) are dealt
// to whichever block finishes first.  It is a kernel of its own, so that the one-shot kernel
// keeps the inlined body.
template <int P, bool SHIELD, bool SPLIT, bool RESAMPLE, bool CON = false, bool PERSIST = false>
__global__ __launch_bounds__(SPLIT ? 512 : 256)
__attribute__((amdgpu_waves_per_eu((SHIELD || RESAMPLE || CON) ? 2
                                   : ((P >= 1 && P <= 4) ? (SPLIT ? 2 : 4) : 3)))) void solve_kernel(
    const InstanceDesc* __restrict__ insts, const BlockDesc* __restrict__ blocks,
    const double* __restrict__ x0_base, const double* __restrict__ Sigma0_base, int extra_shift,
    uint32_t* queue, int nblocks)
{
    if constexpr (!PERSIST) {
        solve_any_block<P, SHIELD, SPLIT, RESAMPLE, CON>(insts, blocks[blockIdx.x], x0_base,
                                                         Sigma0_base, extra_shift);
    } else {
        __shared__ int next_block;
        for (;;) {
            if (threadIdx.x == 0) next_block = (int)atomicAdd(queue, 1u);
            __syncthreads();
            const int b = next_block;
            if (b >= nblocks) break;   // block-uniform
            solve_any_block_call<P, SHIELD, SPLIT, RESAMPLE, CON>(insts, blocks[b], x0_base,
                                                                  Sigma0_base, extra_shift);
            __syncthreads();           // the next entry reuses the block's LDS and next_block
        }
    }
}

__global__ void queue_reset_kernel(uint32_t* queue)
{
    if (threadIdx.x == 0) *queue = 0u;
}

// Resident blocks of one solve-kernel variant on the whole device (the persistent grid).
template <class Kernel>
int resident_grid(Kernel k, int threads, size_t lds)
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, lds) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

// The persistent grid (queue non-null) is built for the plain and split variants only.
template <int P, bool SHIELD, bool SPLIT, bool RESAMPLE, bool CON>
hipError_t launch_variant(const InstanceDesc* inst, const BlockDesc* blocks, int nblocks,
                          size_t lds, const double* x0_base, const double* Sigma0_base,
                          int extra_shift, uint32_t* queue, hipStream_t stream)
{
    const int threads = SPLIT ? 512 : 256;
    if constexpr (!SHIELD && !RESAMPLE && !CON) {
        if (queue) {
            auto kern = solve_kernel<P, SHIELD, SPLIT, RESAMPLE, CON, true>;
            const int resident = resident_grid(kern, threads, lds);
            if (resident <= 0) return hipErrorInvalidValue;
            const int grid = resident < nblocks ? resident : nblocks;
            hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, stream, queue);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, stream, inst, blocks,
                               x0_base, Sigma0_base, extra_shift, queue, nblocks);
            return hipGetLastError();
        }
    } else {
        if (queue) return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((solve_kernel<P, SHIELD, SPLIT, RESAMPLE, CON, false>), dim3(nblocks),
                       dim3(threads), lds, stream, inst, blocks, x0_base, Sigma0_base,
                       extra_shift, nullptr, nblocks);
    return hipGetLastError();
}

template <int P>
hipError_t launch_solve_p(const InstanceDesc* inst, const BlockDesc* blocks, int nblocks,
                          bool shield, bool split, bool resample, bool con, size_t lds,
                          const double* x0_base, const double* Sigma0_base, int extra_shift,
                          uint32_t* queue, hipStream_t stream)
{
    if (con && (shield || resample))
        return launch_variant<P, true, false, true, true>(inst, blocks, nblocks, lds, x0_base,
                                                          Sigma0_base, extra_shift, queue, stream);
    if (con && split)
        return launch_variant<P, false, true, false, true>(inst, blocks, nblocks, lds, x0_base,
                                                           Sigma0_base, extra_shift, queue,
                                                           stream);
    if (con)
        return launch_variant<P, false, false, false, true>(inst, blocks, nblocks, lds, x0_base,
                                                            Sigma0_base, extra_shift, queue,
                                                            stream);
    if (shield && resample)
        return launch_variant<P, true, false, true, false>(inst, blocks, nblocks, lds, x0_base,
                                                           Sigma0_base, extra_shift, queue,
                                                           stream);
    if (shield)
        return launch_variant<P, true, false, false, false>(inst, blocks, nblocks, lds, x0_base,
                                                            Sigma0_base, extra_shift, queue,
                                                            stream);
    if (resample && split)
        return launch_variant<P, false, true, true, false>(inst, blocks, nblocks, lds, x0_base,
                                                           Sigma0_base, extra_shift, queue,
                                                           stream);
    if (resample)
        return launch_variant<P, false, false, true, false>(inst, blocks, nblocks, lds, x0_base,
                                                            Sigma0_base, extra_shift, queue,
                                                            stream);
    if (split)
        return launch_variant<P, false, true, false, false>(inst, blocks, nblocks, lds, x0_base,
                                                            Sigma0_base, extra_shift, queue,
                                                            stream);
    return launch_variant<P, false, false, false, false>(inst, blocks, nblocks, lds, x0_base,
                                                         Sigma0_base, extra_shift, queue, stream);
}

}  // namespace

}  // namespace bss
