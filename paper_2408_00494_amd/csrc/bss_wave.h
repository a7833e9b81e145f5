// bss_wave.h -- wave-level building blocks shared by the solve and merge kernels (gfx950):
// compensated sums, 6x6 factorisations, DPP / swap cross-lane reductions over a lane group, the
// belief scoring of a chunk of records and the block-level log-sum-exp partial.
#pragma once

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
            const double inv = 1.0 / ljj;   // one division per column (FP64 division is long)
            L[j][j] = ljj;
#pragma unroll
            for (int i = j + 1; i < 6; ++i) {
                double acc = A[i][j];
#pragma unroll
                for (int q = 0; q < j; ++q) acc -= L[i][q] * L[j][q];
                L[i][j] = acc * inv;
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

// Orders this wave's LDS accesses around a wave-local exchange: the lanes of a wave run in lockstep
// and their LDS operations complete in program order, so only the compiler must keep the order.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Doubles of LDS that group_sums_lds<., L, N> needs per 256-thread block: each wave holds 64 / L
// groups, each N rows of L + 1 doubles.
template <int N, int L>
constexpr int group_sums_lds_doubles() { return 4 * (64 / L) * N * (L + 1); }

// Sums over the L lanes of each group of N doubles per lane (L = 8, 16 or 32), through the wave's
// own region of `scratch`: one row of L + 1 doubles per value and group (the L lanes' entries, then
// the total).  Lane i of a group adds up rows i, i + L, ... in lane order and stores the totals;
// every lane then reads all N totals, so they are bitwise identical across the group.  The rows'
// odd stride keeps the lanes' accesses on distinct banks.  Every lane of the group takes part.
// The regions are laid out for NCAP >= N values whatever N is, so that calls with different N
// keep every wave inside its own region (waves run apart: one may start its next call while
// another still reads the totals of this one).
template <int N, int L, int NCAP = N>
__device__ __forceinline__ void group_sums_lds(double (&x)[N], double* scratch)
{
    static_assert(L == 8 || L == 16 || L == 32, "group_sums_lds: 8, 16 or 32 lanes");
    static_assert(N <= NCAP, "group_sums_lds: N <= NCAP");
    constexpr int ROW = L + 1;
    const int lane = (int)(threadIdx.x & 63u);
    const int i = lane & (L - 1);
    double* base = scratch + (size_t)(threadIdx.x >> 6) * (64 / L) * NCAP * ROW +
                   (size_t)(lane / L) * NCAP * ROW;
#pragma unroll
    for (int k = 0; k < N; ++k) base[k * ROW + i] = x[k];
    wave_lds_sync();
#pragma unroll
    for (int k0 = 0; k0 < N; k0 += L) {
        const int k = k0 + i;
        if (k < N) {
            const double* row = base + k * ROW;
            double acc = row[0];
#pragma unroll
            for (int q = 1; q < L; ++q) acc += row[q];
            base[k * ROW + L] = acc;
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < N; ++k) x[k] = base[k * ROW + L];
    wave_lds_sync();   // the next call writes the same region
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

// Cost of one belief record: the running cost (eqs. 27-28; times phi_scale on the terminal
// record) plus, on records < T, the control cost (eq. 8); h = the record's barrier value (eq. 33).
// crec: the record's half-space constraint variances, or nullptr where the launch carries none.
__device__ __forceinline__ double record_cost(const ScoreF64& sc, const double* rec, int rec_idx,
                                             int T, const float2* u_row, const double* v,
                                             int vshift, const double* crec, double& h)
{
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
    return q;
}

// C_safe of the transition into a record (eqs. 24-25): C_cbf times the excess of the DCBF
// condition h_t >= (1 - gamma) h_{t-1}; viol (may be null) counts the violating transitions.
__device__ __forceinline__ double transition_cost(const ScoreF64& sc, double h, double h_prev,
                                                 double* viol)
{
    const double excess = -h + (1.0 - sc.gamma) * h_prev;
    if (viol && excess > 0.0) *viol += 1.0;
    return sc.C_cbf * fmax(excess, 0.0);
}

// Score one chunk of belief records, one record per lane of a W-lane group: the record's cost and
// C_safe on the transition into it (record 0 has none).  `h_carry` holds h of the record before
// the chunk and is advanced to the chunk's last record.  Returns this lane's contribution.
__device__ inline double score_chunk(const ScoreF64& sc, const double* rec, int rec_idx, int count,
                                     int lane, int W, int T, const float2* u_row, const double* v,
                                     int vshift, double& h_carry, const double* crec = nullptr,
                                     double* viol = nullptr)
{
    const bool valid = lane < count;
    double part = 0.0;
    double h = 0.0;
    if (valid) part = record_cost(sc, rec, rec_idx, T, u_row, v, vshift, crec, h);
    const double h_left = __shfl(h, lane > 0 ? lane - 1 : 0, W);
    const double h_prev = lane == 0 ? h_carry : h_left;
    if (valid && rec_idx >= 1) part += transition_cost(sc, h, h_prev, viol);
    h_carry = __shfl(h, count - 1, W);
    return part;
}

// Fold n samples (costs S_sh[0..n), controls u_sh[g][T]) into one log-sum-exp partial; nviol is
// the block's count of DCBF violations.
// Must be called by all 256 threads of the block after the inputs are visible in LDS.
__device__ inline void block_partial(int T, int n, const double* S_sh, double* w_sh,
                                     const float2* u_sh, const double* v, int vshift,
                                     double lambda, double nviol, double* out)
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
        out[2 * T + 4] = nviol;
    }
}

}  // namespace

}  // namespace bss
