// bss_solve8.hip -- the solve kernel for the paper's 8-state single-track vehicle with wheel speeds
// (vehicle = 1) on gfx950, and its stand-alone model-step kernel.
//
// x = [vX, vY, r, wF, wR, epsi, eY, s], u = [steer, throttle].  The layout is the 6-state solve's:
// L lanes per control sample (256/L samples per block), P particles per lane in registers, the
// disturbance of each particle quad drawn from three Philox blocks and dealt three normals per
// particle.  Per step every particle takes n_sub explicit-midpoint substeps of the vehicle in
// single precision (magic-formula tires combined by the friction ellipse, wheel speeds, the
// road-aligned kinematics); the belief record of the step -- the mean of the 8 states and the
// unbiased variance of eY -- is reduced across the L lanes in double precision.  The scoring
// (eq. 33 on eY and its spread, the running cost (x - x_g)^T Q (x - x_g) + C_obs [|eY| >= w_T], the
// control cost and C_safe) and the block's log-sum-exp partial follow the particle loop, and the
// merge is the 6-state solve's.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bss_device.h"
#include "bss_internal.h"
#include "bss_wave.h"

namespace bss {

namespace {

constexpr float kInv2PiF = 0.15915494309189535f;

// Magic formula D sin(C atan(B z - E (B z - atan(B z)))) in single precision; the hardware sine
// takes revolutions (|C atan(.)| < C pi / 2 keeps it within one revolution).
__device__ __forceinline__ float magic_f32(const Car8F32& c, float z)
{
    const float bz = c.B * z;
    const float a1 = atan_f32(bz);
    const float a2 = atan_f32(fmaf(-c.E, bz - a1, bz));
    return c.D * __builtin_amdgcn_sinf(c.C * a2 * kInv2PiF);
}

// Quantities of one (sample, step) shared by its particles.
struct Step8 {
    float sd, cd;      // sine and cosine of the steering angle
    float drive;       // throttle T_max / Iw
};

__device__ __forceinline__ Step8 make_step8(const Car8F32& c, float steer, float throttle)
{
    Step8 s;
    const float rev = steer * kInv2PiF;   // |steer| < pi
    s.sd = __builtin_amdgcn_sinf(rev);
    s.cd = __builtin_amdgcn_cosf(rev);
    s.drive = throttle * c.Tmax_Iw;
    return s;
}

// Vector field of the 8-state vehicle; x[7] is the path coordinate relative to the estimate's,
// s0rev the estimate's sin(4 pi s / L) phase in revolutions (reduced to [-1/2, 1/2]).
__device__ __forceinline__ void car8_field(const Car8F32& c, const Step8& st, float s0rev,
                                           const float* x, float* dx)
{
    const float vX = x[0], vY = x[1], r = x[2], wF = x[3], wR = x[4], ep = x[5], eY = x[6];
    const float vyb = fmaf(c.lf, r, vY);
    const float vxf = fmaf(vX, st.cd, vyb * st.sd);
    const float vyf = fmaf(vyb, st.cd, -vX * st.sd);
    const float vyr = fmaf(-c.lr, r, vY);
    const float inf = __builtin_amdgcn_rcpf(fmaxf(vxf, c.v_min));
    const float inr = __builtin_amdgcn_rcpf(fmaxf(vX, c.v_min));
    const float slf = fmaf(c.Rw, wF, -vxf) * inf;
    const float slr = fmaf(c.Rw, wR, -vX) * inr;
    const float alf = -atan_f32(vyf * inf);
    const float alr = -atan_f32(vyr * inr);
    // pure-slip forces, then the friction ellipse (the lateral force takes what the longitudinal
    // one leaves)
    const float fxf = c.muFzf * magic_f32(c, slf);
    const float fy0f = c.muFzf * magic_f32(c, alf);
    const float fxr = c.muFzr * magic_f32(c, slr);
    const float fy0r = c.muFzr * magic_f32(c, alr);
    const float qf = fxf * c.inv_fmaxf, qr = fxr * c.inv_fmaxr;
    const float fyf = fy0f * __builtin_amdgcn_sqrtf(fmaxf(fmaf(-qf, qf, 1.0f), 0.0f));
    const float fyr = fy0r * __builtin_amdgcn_sqrtf(fmaxf(fmaf(-qr, qr, 1.0f), 0.0f));
    const float fxb = fmaf(fxf, st.cd, fmaf(-fyf, st.sd, fxr));
    const float fyfront = fmaf(fxf, st.sd, fyf * st.cd);
    dx[0] = fmaf(r, vY, fxb * c.inv_m);
    dx[1] = fmaf(-r, vX, (fyfront + fyr) * c.inv_m);
    dx[2] = fmaf(c.lf, fyfront, -c.lr * fyr) * c.inv_Iz;
    dx[3] = -c.Rw_Iw * fxf;
    dx[4] = fmaf(-c.Rw_Iw, fxr, st.drive);
    // road-aligned kinematics with kappa(s) = kappa0 (1 + a sin(4 pi s / L))
    float rev = fmaf(x[7], c.s_rev, s0rev);
    rev = rev - rintf(rev);
    const float kap = c.kappa0 * fmaf(c.kappa_amp, __builtin_amdgcn_sinf(rev), 1.0f);
    const float erev = ep * kInv2PiF;    // heading errors stay far below a revolution
    const float se = __builtin_amdgcn_sinf(erev), ce = __builtin_amdgcn_cosf(erev);
    const float sdot = fmaf(vX, ce, -vY * se) * __builtin_amdgcn_rcpf(fmaf(-kap, eY, 1.0f));
    dx[5] = fmaf(-kap, sdot, r);
    dx[6] = fmaf(vX, se, vY * ce);
    dx[7] = sdot;
}

// One control period of Q particles: n_sub midpoint substeps (the particles' evaluations in one
// straight-line block per stage, so the compiler interleaves them).
template <int Q>
__device__ __forceinline__ void car8_period(const Car8F32& c, const Step8& st, float s0rev,
                                            float (*x)[8])
{
    for (int i = 0; i < c.n_sub; ++i) {
        float k1[Q][8], xm[Q][8], k2[Q][8];
#pragma unroll
        for (int q = 0; q < Q; ++q) car8_field(c, st, s0rev, x[q], k1[q]);
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int j = 0; j < 8; ++j) xm[q][j] = fmaf(c.half_h, k1[q][j], x[q][j]);
#pragma unroll
        for (int q = 0; q < Q; ++q) car8_field(c, st, s0rev, xm[q], k2[q]);
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int j = 0; j < 8; ++j) x[q][j] = fmaf(c.h, k2[q][j], x[q][j]);
    }
}

// Barrier eq. 33 of an 8-state record (mean eY in rec[6], its variance in rec[8]).
__device__ __forceinline__ double barrier8(const ScoreF64& sc, const double* rec)
{
    const double margin = fmax(sc.half_width - sc.nu * sqrt(fmax(rec[8], 0.0)), 0.0);
    return margin * margin - rec[6] * rec[6];
}

// Score one chunk of 8-state records, one per lane of a W-lane group (as score_chunk).
__device__ inline double score_chunk8(const ScoreF64& sc, const double* rec, int rec_idx,
                                      int count, int lane, int W, int T, const float2* u_row,
                                      const double* v, int vshift, double& h_carry, double& viol)
{
    const bool valid = lane < count;
    double part = 0.0, h = 0.0;
    if (valid) {
        const double dv = rec[0] - sc.v_goal;
        double q = sc.q_vx * dv * dv + sc.q_vy * rec[1] * rec[1] + sc.q_r * rec[2] * rec[2] +
                   sc.q_epsi * rec[5] * rec[5] + sc.q_ey * rec[6] * rec[6];
        if (fabs(rec[6]) >= sc.half_width) q += sc.C_obs;
        if (rec_idx == T) {
            q *= sc.phi_scale;
        } else {
            const float2 ut = u_row[rec_idx];
            const int r = vrow(rec_idx, vshift, T);
            q += sc.gamma_u * (v[2 * r] * sc.inv_var0 * (double)ut.x +
                               v[2 * r + 1] * sc.inv_var1 * (double)ut.y);
        }
        h = barrier8(sc, rec);
        part = q;
    }
    const double h_left = __shfl(h, lane > 0 ? lane - 1 : 0, W);
    const double h_prev = lane == 0 ? h_carry : h_left;
    if (valid && rec_idx >= 1) {
        const double excess = -h + (1.0 - sc.gamma) * h_prev;
        part += sc.C_cbf * fmax(excess, 0.0);
        if (excess > 0.0) viol += 1.0;
    }
    h_carry = __shfl(h, count - 1, W);
    return part;
}

template <int P, int L>
__device__ __forceinline__ void solve8_block(const InstanceDesc& d, const BlockDesc bd,
                                             const double* __restrict__ x0_base, int extra_shift)
{
    constexpr int log2L = L == 8 ? 3 : (L == 16 ? 4 : (L == 32 ? 5 : 6));
    constexpr int groups = 256 >> log2L;
    const int T = d.T, M = d.M;
    const int vshift = d.vshift + extra_shift;
    const double* __restrict__ v = d.v[d.cur];
    extern __shared__ double smem[];
    double* S_sh = smem;
    double* w_sh = S_sh + groups;
    float2* u_sh = reinterpret_cast<float2*>(w_sh + groups);
    const int q = (int)threadIdx.x;
    const int g = q >> log2L;
    const int j = q & (L - 1);
    const int k = bd.k0 + g;
    const bool active = k < d.K;
    float2* us = u_sh + g * T;
    double* mom_k = d.mom + (size_t)(active ? k : 0) * (T + 1) * 9;
    const uint32_t s = d.solve_index;
    const uint32_t key0 = d.key0, key1 = d.key1;
    const double* x0p = x0_base + 8 * d.x0_index;

    // control samples u = clip(v + eps) (tag 0), lane-parallel over t
    if (active) {
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
            if (d.u) reinterpret_cast<float2*>(d.u)[(size_t)k * T + t] = us[t];
        }
    }
    __syncthreads();

    if (active) {
        double x0[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) x0[i] = x0p[i];
        const Car8F32 car = d.car8;
        // the path coordinate is carried relative to the estimate's; its curvature phase
        const double ph = x0[7] * (double)car.s_rev;
        const float s0rev = (float)(ph - rint(ph));
        float x[P][8];
#pragma unroll
        for (int p = 0; p < P; ++p) {
#pragma unroll
            for (int i = 0; i < 7; ++i) x[p][i] = (float)x0[i];
            x[p][7] = 0.0f;
        }
        if (j == 0) {
#pragma unroll
            for (int i = 0; i < 8; ++i) mom_k[i] = x0[i];
            mom_k[8] = 0.0;
        }
        const uint32_t c3w = rng_word3(kTagW, s);
        const uint64_t pk = (uint64_t)kPhiloxM1 * (d.crn ? 0u : (uint32_t)k);
        const uint32_t hk = (uint32_t)(pk >> 32), lk = (uint32_t)pk;
        constexpr int NB = noise_blocks<P>();
        PhiloxParticle pb[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i)
            pb[i] = philox_particle(noise_block_word<P, L>(j, i), hk, key0, key1);
        const float sw0 = d.sig_w0, sw1 = d.sig_w1, sw2 = d.sig_w2;
        const double invM = 1.0 / (double)M;
        const double invM1 = M > 1 ? 1.0 / (double)(M - 1) : 0.0;

        for (int t = 0; t < T; ++t) {
            const float2 uu = us[t];
            const Step8 st = make_step8(car, uu.x, uu.y);
            // two particles at a time: their stages interleave, and the registers of the
            // midpoint stages of more would not fit beside the other particles' states
            constexpr int Q = P < 2 ? P : 2;
#pragma unroll
            for (int p0 = 0; p0 < P; p0 += Q) car8_period<Q>(car, st, s0rev, x + p0);
            const PhiloxStep ps = philox_step((uint32_t)t, c3w, lk, key0, key1);
            NoiseDealer<P> deal{ps, pb, key0, key1, j, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int p = 0; p < P; ++p) {
                float w0, w1, w2;
                deal.next(p, w0, w1, w2);
                x[p][0] = fmaf(sw0, w0, x[p][0]);
                x[p][1] = fmaf(sw1, w1, x[p][1]);
                x[p][2] = fmaf(sw2, w2, x[p][2]);
            }
            // FP64 sums of the lane's particles: the 8 states, and eY shifted by particle 0's
            // (lane 0 of the group) with its square
            const double ref = (double)group_first(x[0][6], L);
            double sm[8], sq = 0.0, se = 0.0;
#pragma unroll
            for (int i = 0; i < 8; ++i) sm[i] = 0.0;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (particle_of<P, L>(j, p) < M) {
#pragma unroll
                    for (int i = 0; i < 8; ++i) sm[i] += (double)x[p][i];
                    const double e = (double)x[p][6] - ref;
                    se += e;
                    sq = fma(e, e, sq);
                }
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) sm[i] = group_sum(sm[i], L);
            se = group_sum(se, L);
            sq = group_sum(sq, L);
            if (j == ((t + 1) & (L - 1))) {
                double* rec = mom_k + (size_t)(t + 1) * 9;
#pragma unroll
                for (int i = 0; i < 7; ++i) rec[i] = sm[i] * invM;
                rec[7] = x0[7] + sm[7] * invM;
                rec[8] = (sq - se * (se * invM)) * invM1;
            }
        }
    }
    // score the belief trajectory, L records at a time
    __threadfence_block();
    __syncthreads();
    double S_part = 0.0, V_part = 0.0;
    if (active) {
        double h_carry = 0.0;
        for (int base = 0; base <= T; base += L) {
            const int count = min(L, T + 1 - base);
            const int rec = base + min(j, count - 1);
            S_part += score_chunk8(d.sc, mom_k + (size_t)rec * 9, base + j, count, j, L, T, us,
                                   v, vshift, h_carry, V_part);
        }
    }
    const double S_k = group_sum(S_part, L);
    const double V_k = group_sum(V_part, L);
    __shared__ double viol_sh[32];           // DCBF violations per group (at most 32 groups)
    if (j == 0) {
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

template <int P>
__global__ __launch_bounds__(256) void solve8_kernel(const InstanceDesc* __restrict__ insts,
                                                     const BlockDesc* __restrict__ blocks,
                                                     const double* __restrict__ x0_base,
                                                     int extra_shift)
{
    const BlockDesc bd = blocks[blockIdx.x];
    const InstanceDesc& d = insts[bd.inst];
    switch (d.lanes) {
    case 8: solve8_block<P, 8>(d, bd, x0_base, extra_shift); break;
    case 16: solve8_block<P, 16>(d, bd, x0_base, extra_shift); break;
    case 32: solve8_block<P, 32>(d, bd, x0_base, extra_shift); break;
    default: solve8_block<P, 64>(d, bd, x0_base, extra_shift); break;
    }
}

__global__ void model_step8_kernel(Car8F32 car, const float* x, const float* u, float* xn,
                                   int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float st[1][8];
#pragma unroll
    for (int j = 0; j < 8; ++j) st[0][j] = x[8 * i + j];
    // absolute path coordinate: phase from s itself, relative coordinate 0
    const double ph = (double)st[0][7] * (double)car.s_rev;
    const float s0rev = (float)(ph - rint(ph));
    const float s_abs = st[0][7];
    st[0][7] = 0.0f;
    const Step8 stp = make_step8(car, u[2 * i], u[2 * i + 1]);
    car8_period<1>(car, stp, s0rev, st);
#pragma unroll
    for (int j = 0; j < 7; ++j) xn[8 * i + j] = st[0][j];
    xn[8 * i + 7] = s_abs + st[0][7];
}

}  // namespace

hipError_t launch_solve8(const InstanceDesc* inst, const BlockDesc* blocks, int nblocks, int ppl,
                         size_t lds, const double* x0_base, int extra_shift, hipStream_t stream)
{
    if (nblocks <= 0) return hipSuccess;
    const dim3 g(nblocks), b(256);
    switch (ppl) {
    case 1:
        hipLaunchKernelGGL(solve8_kernel<1>, g, b, lds, stream, inst, blocks, x0_base, extra_shift);
        break;
    case 2:
        hipLaunchKernelGGL(solve8_kernel<2>, g, b, lds, stream, inst, blocks, x0_base, extra_shift);
        break;
    case 4:
        hipLaunchKernelGGL(solve8_kernel<4>, g, b, lds, stream, inst, blocks, x0_base, extra_shift);
        break;
    case 8:
        hipLaunchKernelGGL(solve8_kernel<8>, g, b, lds, stream, inst, blocks, x0_base, extra_shift);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_model_step8(const Car8F32& car, const float* x, const float* u, float* xn,
                              int64_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(model_step8_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       car, x, u, xn, n);
    return hipGetLastError();
}

}  // namespace bss
