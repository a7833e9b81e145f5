// bss_device.h -- device-side building blocks of the BSS-MPPI solve (gfx950).
//
//  * Philox4x32-10 and Box-Muller normals (the random-number contract: counter words
//    (t or block, particle m, sample k, (tag << 28) | solve index), key (lo32 seed, hi32 seed)).
//  * the single-precision car vector field used by the particle integrator;
//  * double-precision versions of the model, the track signed distance, the belief-space barrier
//    and the running cost used per (sample, step).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bss_internal.h"

namespace bss {

// ------------------------------------------------------------------------------------------------
// random numbers
// ------------------------------------------------------------------------------------------------
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

constexpr uint32_t kTagEps = 0u;
constexpr uint32_t kTagW = 1u;
constexpr uint32_t kTagInit = 2u;
constexpr uint32_t kTagResample0 = 4u;   // normals xi_0..2 of a Gaussian re-sampling draw
constexpr uint32_t kTagResample1 = 5u;   // normals xi_3..5

__device__ __forceinline__ uint32_t rng_word3(uint32_t tag, uint32_t s)
{
    return (tag << 28) | (s & 0x0FFFFFFFu);
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);   // a ^ b ^ c in one instruction
}

// One Philox round on (c0..c3) with round key (k0, k1).
__device__ __forceinline__ void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                             uint32_t k0, uint32_t k1)
{
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
}

// Ten Philox rounds on (c0..c3) in place; the round key starts at (k0, k1) and advances by the
// two Weyl constants after each round.
__device__ __forceinline__ void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                         uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        philox_round(c0, c1, c2, c3, k0, k1);
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
}

// The disturbance stream uses counters (t, m, k, w3): over a sample's horizon only t changes.
// The first round's products M0 t and M1 k, and the second round's product of word 0, are
// therefore shared: per particle (m, k) two words are fixed for the whole horizon, per step t
// three words are common to all particles of the sample.  philox10_tail finishes the remaining
// eight rounds; the result equals philox10 on (t, m, k, w3) bit for bit.
struct PhiloxParticle {
    uint32_t ph;   // hi(M0 a0) ^ (k1 + W1), with a0 = hi(M1 k) ^ m ^ k0
    uint32_t pl;   // lo(M0 a0)
};

struct PhiloxStep {
    uint32_t b0;   // hi(M1 a2) ^ lo(M1 k) ^ (k0 + W0), with a2 = hi(M0 t) ^ w3 ^ k1
    uint32_t b1;   // lo(M1 a2)
    uint32_t a3;   // lo(M0 t)
};

__device__ __forceinline__ PhiloxParticle philox_particle(uint32_t m, uint32_t hk, uint32_t k0,
                                                          uint32_t k1)
{
    const uint32_t a0 = xor3(hk, m, k0);
    const uint64_t p = (uint64_t)kPhiloxM0 * a0;
    PhiloxParticle r;
    r.ph = (uint32_t)(p >> 32) ^ (k1 + kPhiloxW1);
    r.pl = (uint32_t)p;
    return r;
}

__device__ __forceinline__ PhiloxStep philox_step(uint32_t t, uint32_t w3, uint32_t lk,
                                                  uint32_t k0, uint32_t k1)
{
    const uint64_t p0 = (uint64_t)kPhiloxM0 * t;
    const uint32_t a2 = xor3((uint32_t)(p0 >> 32), w3, k1);
    const uint64_t p1 = (uint64_t)kPhiloxM1 * a2;
    PhiloxStep r;
    r.b0 = xor3((uint32_t)(p1 >> 32), lk, k0 + kPhiloxW0);
    r.b1 = (uint32_t)p1;
    r.a3 = (uint32_t)p0;
    return r;
}

// rounds 3..10 from the shared first two rounds; outputs the four words in (c0..c3)
__device__ __forceinline__ void philox10_tail(const PhiloxStep& st, const PhiloxParticle& pp,
                                              uint32_t k0, uint32_t k1, uint32_t& c0,
                                              uint32_t& c1, uint32_t& c2, uint32_t& c3)
{
    c0 = st.b0;
    c1 = st.b1;
    c2 = pp.ph ^ st.a3;
    c3 = pp.pl;
    k0 += 2u * kPhiloxW0;
    k1 += 2u * kPhiloxW1;
#pragma unroll
    for (int i = 2; i < 10; ++i) {
        philox_round(c0, c1, c2, c3, k0, k1);
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
}

// ((r >> 9) + 1/2) * 2^-23 without a conversion: the bit pattern (r >> 9) | 0x3F800000 is
// 1 + (r >> 9) 2^-23, and subtracting 1 - 2^-24 is exact (Sterbenz).
__device__ __forceinline__ float uniform01(uint32_t r)
{
    return __uint_as_float((r >> 9) | 0x3F800000u) - 0.999999940395355224609375f;
}

// Box-Muller on one pair of words: rho = sqrt(-2 ln u_a), angle 2 pi u_b.  The hardware log is
// base 2 and the hardware sine/cosine take their argument in revolutions.
__device__ __forceinline__ float bm_radius(uint32_t ra)
{
    const float la = __builtin_amdgcn_logf(uniform01(ra));               // log2(u)
    return __builtin_amdgcn_sqrtf(-1.3862943611198906f * la);            // -2 ln 2 log2(u)
}

__device__ __forceinline__ void bm_pair(uint32_t ra, uint32_t rb, float& z0, float& z1)
{
    const float rho = bm_radius(ra);
    const float ub = uniform01(rb);
    z0 = rho * __builtin_amdgcn_cosf(ub);
    z1 = rho * __builtin_amdgcn_sinf(ub);
}

__device__ __forceinline__ float bm_cos(uint32_t ra, uint32_t rb)
{
    return bm_radius(ra) * __builtin_amdgcn_cosf(uniform01(rb));
}

// ---- disturbance normals, dealt from particle quads ----
// Particle quad q = m / 4 owns the three Philox blocks whose counter word 1 is 3q + b (b = 0, 1,
// 2).  Block b yields the normals 4b .. 4b + 3 (Box-Muller on words (0, 1), then on (2, 3)); the
// twelve are dealt three per particle in order, particle 4q + i taking normals 3i .. 3i + 2.  So
// particle i of a quad reads block i's first normals and what block i - 1 left over.
//
// Placement of particles in a group of L lanes with P particles per lane: with four or more, a
// lane holds whole quads (slots 4h .. 4h + 3 are quad j + h L); with one or two, the 4 / P lanes
// of an aligned lane quad share one particle quad (slot p of lane j is particle P j + p).
template <int P, int L>
__device__ __forceinline__ int particle_of(int j, int p)
{
    return P >= 4 ? 4 * (j + L * (p >> 2)) + (p & 3) : P * j + p;
}

// Philox blocks a lane draws per step, and the counter word 1 of its block i.  With one particle
// per lane, lane i of a lane quad draws block min(i, 2) (lanes 2 and 3 draw the same block).
template <int P>
constexpr int noise_blocks()
{
    return P >= 4 ? 3 * (P / 4) : (P == 2 ? 2 : 1);
}

template <int P, int L>
__device__ __forceinline__ uint32_t noise_block_word(int j, int i)
{
    if (P >= 4) return (uint32_t)(3 * (j + L * (i / 3)) + i % 3);
    if (P == 2) return (uint32_t)(3 * (j >> 1) + (j & 1) + i);
    return (uint32_t)(3 * (j >> 2) + ((j & 3) < 2 ? (j & 3) : 2));
}

// Deals the disturbance normals of the lane's particles slot by slot.  Call next() for slots
// 0, 1, ..., P - 1 in order (the calls are unrolled, so the carried normals stay in registers):
// each block is drawn and transformed when its first particle needs it.
template <int P>
struct NoiseDealer {
    const PhiloxStep& ps;
    const PhiloxParticle* pb;     // the lane's noise_blocks<P>() per-block Philox parts
    uint32_t key0, key1;
    int j;                        // lane in the group
    float c0, c1, c2;             // normals left over by the previous block of the quad

    __device__ __forceinline__ void block(int bi, float* z) const
    {
        uint32_t r0, r1, r2, r3;
        philox10_tail(ps, pb[bi], key0, key1, r0, r1, r2, r3);
        bm_pair(r0, r1, z[0], z[1]);
        bm_pair(r2, r3, z[2], z[3]);
    }

    __device__ __forceinline__ void next(int p, float& w0, float& w1, float& w2)
    {
        if constexpr (P >= 4) {
            const int i = p & 3, h = p >> 2;
            float z[4];
            if (i < 3) block(3 * h + i, z);
            if (i == 0) {
                w0 = z[0]; w1 = z[1]; w2 = z[2];
                c0 = z[3];
            } else if (i == 1) {
                w0 = c0; w1 = z[0]; w2 = z[1];
                c0 = z[2]; c1 = z[3];
            } else if (i == 2) {
                w0 = c0; w1 = c1; w2 = z[0];
                c0 = z[1]; c1 = z[2]; c2 = z[3];
            } else {
                w0 = c0; w1 = c1; w2 = c2;
            }
        } else if constexpr (P == 2) {
            // lane half e = j & 1 of its quad holds particles 2e, 2e + 1 and draws blocks e and
            // e + 1 (A and B): e = 0 takes (A0 A1 A2) (A3 B0 B1), e = 1 takes (A2 A3 B0)
            // (B1 B2 B3); the pair that only one half needs is selected before its transform
            if (p == 0) {
                uint32_t a[4], b[4];
                philox10_tail(ps, pb[0], key0, key1, a[0], a[1], a[2], a[3]);
                philox10_tail(ps, pb[1], key0, key1, b[0], b[1], b[2], b[3]);
                const bool e = (j & 1) != 0;
                float a2, a3, b0, b1, x0, x1;
                bm_pair(a[2], a[3], a2, a3);
                bm_pair(b[0], b[1], b0, b1);
                bm_pair(e ? b[2] : a[0], e ? b[3] : a[1], x0, x1);
                w0 = e ? a2 : x0; w1 = e ? a3 : x1; w2 = e ? b0 : a2;
                c0 = e ? b1 : a3; c1 = e ? x0 : b0; c2 = e ? x1 : b1;
            } else {
                w0 = c0; w1 = c1; w2 = c2;
            }
        } else {
            // lane i of its lane quad holds particle i and drew block min(i, 2); lane 1 needs
            // lane 0's fourth normal, lane 2 lane 1's third and fourth (quad_perm [0, 0, 1, 3])
            float z[4];
            block(0, z);
            constexpr int kPerm = 0xD0;
            const float pz2 = __int_as_float(
                __builtin_amdgcn_mov_dpp(__float_as_int(z[2]), kPerm, 0xf, 0xf, true));
            const float pz3 = __int_as_float(
                __builtin_amdgcn_mov_dpp(__float_as_int(z[3]), kPerm, 0xf, 0xf, true));
            const int i = j & 3;
            w0 = i == 0 ? z[0] : (i == 1 ? pz3 : (i == 2 ? pz2 : z[1]));
            w1 = i == 0 ? z[1] : (i == 1 ? z[0] : (i == 2 ? pz3 : z[2]));
            w2 = i == 0 ? z[2] : (i == 1 ? z[1] : (i == 2 ? z[0] : z[3]));
        }
    }
};

// ------------------------------------------------------------------------------------------------
// single-precision car model
// ------------------------------------------------------------------------------------------------
// atan on [-1, 1]: atan(z) = z + z^3 P(z^2) with a degree-7 polynomial P fitted for relative
// error (max ~1e-7).
__device__ __forceinline__ float atan_poly(float z)
{
    const float z2 = z * z;
    float p = 0.0029182303696870804f;
    p = fmaf(p, z2, -0.016349468380212784f);
    p = fmaf(p, z2, 0.04316648095846176f);
    p = fmaf(p, z2, -0.07546935230493546f);
    p = fmaf(p, z2, 0.10662780702114105f);
    p = fmaf(p, z2, -0.1421002447605133f);
    p = fmaf(p, z2, 0.1999361664056778f);
    p = fmaf(p, z2, -0.333331435918808f);
    return fmaf(z * z2, p, z);
}

// atan on the whole line: |x| > 1 is folded through atan(x) = sign(x) pi/2 - atan(1/x).
__device__ __forceinline__ float atan_f32(float x)
{
    const float ax = fabsf(x);
    const float z = fminf(ax, 1.0f) * __builtin_amdgcn_rcpf(fmaxf(ax, 1.0f));
    float r = atan_poly(z);
    r = ax > 1.0f ? 1.5707963267948966f - r : r;
    return copysignf(r, x);
}

// min(max(x, lo), hi) for lo <= hi as one median-of-three: a NaN x gives lo, as the min/max pair
// does (the instruction returns the minimum of the other two inputs then), and no operand needs
// the quieting move that the min/max pair gets for values the compiler cannot prove canonical.
__device__ __forceinline__ float clamp_f32(float x, float lo, float hi)
{
    return __builtin_amdgcn_fmed3f(x, lo, hi);
}

// Quantities of one (sample, step) that every particle of the sample shares.
struct StepF32 {
    float steer, accel;
    float sd, cd;              // sin / cos of the steering angle
    float kz_lf_cd;            // (m/Iz) lf cos(steer)
    float kz_lr;               // (m/Iz) lr
};

__device__ __forceinline__ StepF32 make_step(const CarF32& car, float steer, float accel)
{
    StepF32 s;
    s.steer = steer;
    s.accel = accel;
    // |steer| <= steer_max < pi, so the hardware sine/cosine (argument in revolutions) is used
    const float rev = steer * 0.15915494309189535f;
    s.sd = __builtin_amdgcn_sinf(rev);
    s.cd = __builtin_amdgcn_cosf(rev);
    s.kz_lf_cd = car.m_Iz * car.lf * s.cd;
    s.kz_lr = car.m_Iz * car.lr;
    return s;
}

// Vector field of the velocity/heading part for P particles of one sample at once (arrays of P
// registers after inlining).  `rev` is the
// heading in revolutions (the global position derivative needs sin/cos of the heading).  Outputs:
// dX, dY, dvx, dvy, dr (dpsi = r).  The slip-angle arctangents skip the |x| > 1 folding when no
// argument of any of the P particles in any lane of the wave needs it (the usual case: the
// body-frame lateral speeds are small against max(vx, v_min)); both forms give the same value
// on [-1, 1], so the result does not depend on the branch.  Deciding once for all P particles
// keeps their evaluations in one straight-line block, where the compiler interleaves them.
template <int P>
__device__ __forceinline__ void car_field_f32_n(const CarF32& car, const StepF32& st,
                                                const float* rev, const float* vx,
                                                const float* vy, const float* r, float* dX,
                                                float* dY, float* dvx, float* dvy, float* dr)
{
    float xa[P], xb[P];
    float big = 0.0f;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const float inv_vx = __builtin_amdgcn_rcpf(clamp_f32(vx[p], car.v_min, INFINITY));
        xa[p] = fmaf(car.lf, r[p], vy[p]) * inv_vx;
        xb[p] = fmaf(-car.lr, r[p], vy[p]) * inv_vx;
        big = fmaxf(big, fmaxf(fabsf(xa[p]), fabsf(xb[p])));
    }
    float atf[P], atr[P];
    if (__all(big <= 1.0f)) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            atf[p] = atan_poly(xa[p]);
            atr[p] = atan_poly(xb[p]);
        }
    } else {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            atf[p] = atan_f32(xa[p]);
            atr[p] = atan_f32(xb[p]);
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const float af = st.steer - atf[p];
        const float ar = -atr[p];
        const float fF = clamp_f32(car.cf_m * af, -car.fF_max, car.fF_max);   // F_f / m
        const float fR = clamp_f32(car.cr_m * ar, -car.fR_max, car.fR_max);   // F_r / m
        const float rr = rev[p] - rintf(rev[p]);
        const float sp = __builtin_amdgcn_sinf(rr);
        const float cp = __builtin_amdgcn_cosf(rr);
        dX[p] = fmaf(vx[p], cp, -vy[p] * sp);
        dY[p] = fmaf(vx[p], sp, vy[p] * cp);
        dvx[p] = fmaf(-fF, st.sd, fmaf(vy[p], r[p], st.accel));
        dvy[p] = fmaf(fF, st.cd, fmaf(-vx[p], r[p], fR));
        dr[p] = fmaf(fF, st.kz_lf_cd, -st.kz_lr * fR);
    }
}

// One particle.
__device__ __forceinline__ void car_field_f32(const CarF32& car, const StepF32& st, float rev,
                                              float vx, float vy, float r, float& dX, float& dY,
                                              float& dvx, float& dvy, float& dr)
{
    float a[1] = {rev}, b[1] = {vx}, c[1] = {vy}, e[1] = {r};
    float o0[1], o1[1], o2[1], o3[1], o4[1];
    car_field_f32_n<1>(car, st, a, b, c, e, o0, o1, o2, o3, o4);
    dX = o0[0];
    dY = o1[0];
    dvx = o2[0];
    dvy = o3[0];
    dr = o4[0];
}

// ------------------------------------------------------------------------------------------------
// double-precision model, track geometry, barrier and cost
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ double clampd(double x, double lo, double hi)
{
    return fmin(fmax(x, lo), hi);
}

// sin and cos of an angle |x| <= pi/2 by their Taylor series through x^23 and x^22 (truncation
// below 2e-18 there, so the results are the correctly rounded values to within an ulp); wider
// angles take the library routine.  Steering angles, bounded by steer_max, use this.
__device__ __forceinline__ void sincos_small_f64(double x, double* s, double* c)
{
    if (!(fabs(x) <= 1.5707963267948966)) {
        sincos(x, s, c);
        return;
    }
    const double x2 = x * x;
    // sin x = x (1 + sum_n (-1)^n x^2n / (2n+1)!), cos x = 1 + sum_n (-1)^n x^2n / (2n)!,
    // n = 1 .. 11, by Horner's rule in x^2
    double ps = -3.868170170630684e-23;
    ps = fma(ps, x2, 1.9572941063391263e-20);
    ps = fma(ps, x2, -8.22063524662433e-18);
    ps = fma(ps, x2, 2.8114572543455206e-15);
    ps = fma(ps, x2, -7.647163731819816e-13);
    ps = fma(ps, x2, 1.6059043836821613e-10);
    ps = fma(ps, x2, -2.505210838544172e-08);
    ps = fma(ps, x2, 2.7557319223985893e-06);
    ps = fma(ps, x2, -0.0001984126984126984);
    ps = fma(ps, x2, 0.008333333333333333);
    ps = fma(ps, x2, -0.16666666666666666);
    *s = fma(x * x2, ps, x);
    double pc = -8.896791392450574e-22;
    pc = fma(pc, x2, 4.110317623312165e-19);
    pc = fma(pc, x2, -1.5619206968586225e-16);
    pc = fma(pc, x2, 4.779477332387385e-14);
    pc = fma(pc, x2, -1.1470745597729725e-11);
    pc = fma(pc, x2, 2.08767569878681e-09);
    pc = fma(pc, x2, -2.755731922398589e-07);
    pc = fma(pc, x2, 2.48015873015873e-05);
    pc = fma(pc, x2, -0.001388888888888889);
    pc = fma(pc, x2, 0.041666666666666664);
    pc = fma(pc, x2, -0.5);
    *c = fma(x2, pc, 1.0);
}

__device__ inline void car_deriv_f64(const ScoreF64& p, const double* x, double steer,
                                     double accel, double* dx)
{
    const double psi = x[2], vx = x[3], vy = x[4], r = x[5];
    // one reciprocal for both slip angles; force limits, 1/m and 1/Iz come precomputed (FP64
    // division is a long instruction sequence on this GPU)
    const double inv_vxs = 1.0 / fmax(vx, p.v_min);
    const double af = steer - atan((vy + p.lf * r) * inv_vxs);
    const double ar = -atan((vy - p.lr * r) * inv_vxs);
    const double Ff = clampd(p.Cf * af, -p.Ffm, p.Ffm);
    const double Fr = clampd(p.Cr * ar, -p.Frm, p.Frm);
    double sp, cp, sd, cd;
    sincos(psi, &sp, &cp);
    sincos_small_f64(steer, &sd, &cd);
    dx[0] = vx * cp - vy * sp;
    dx[1] = vx * sp + vy * cp;
    dx[2] = r;
    dx[3] = accel + vy * r - Ff * sd * p.inv_m;
    dx[4] = (Ff * cd + Fr) * p.inv_m - vx * r;
    dx[5] = (p.lf * Ff * cd - p.lr * Fr) * p.inv_Iz;
}

// explicit midpoint step of the noise-free model in double precision
__device__ inline void car_step_f64(const ScoreF64& p, const double* x, double steer, double accel,
                                    double* xn)
{
    double k1[6], xm[6], k2[6];
    car_deriv_f64(p, x, steer, accel, k1);
#pragma unroll
    for (int i = 0; i < 6; ++i) xm[i] = x[i] + 0.5 * p.dt * k1[i];
    car_deriv_f64(p, xm, steer, accel, k2);
#pragma unroll
    for (int i = 0; i < 6; ++i) xn[i] = x[i] + p.dt * k2[i];
}

// Nearest point of the ellipse (e0 >= e1) to (y0, y1) in the first quadrant.  Parametrising the
// nearest point as c0 = r0 y0 / (s + r0) e0-scaled, c1 = y1 / (s + 1) (r0 = (e0/e1)^2) turns the
// problem into the root of the convex decreasing F(s) = (r0 z0/(s+r0))^2 + (z1/(s+1))^2 - 1 on
// (z1 - 1, |(r0 z0, z1)| - 1]; it is found by Newton's method safeguarded by that bracket,
// started from the first-order distance estimate.  Newton converges quadratically, so once a
// Newton step (not a bisection) is below 1e-8 of the scale the iterate is accurate to the last
// bits and the loop ends there (3.2 iterations on average for points within 2 m of a 30 m x 20 m
// track, against 4.9 when the loop waited for a step below 1e-16).
// The divisions by the semi-axes are multiplications by the precomputed reciprocals.
__device__ inline void ellipse_nearest_q1(const EllipseF64& E, double y0, double y1, double* c0,
                                          double* c1)
{
    const double e0 = E.e0, e1 = E.e1;
    if (y1 > 0.0) {
        if (y0 > 0.0) {
            const double z0 = y0 * E.inv_e0, z1 = y1 * E.inv_e1;
            const double g = z0 * z0 + z1 * z1 - 1.0;
            if (g != 0.0) {
                const double r0 = E.r0;
                const double n0 = r0 * z0;
                double lo = z1 - 1.0;
                double hi = g < 0.0 ? 0.0 : sqrt(n0 * n0 + z1 * z1) - 1.0;
                // first-order signed distance d ~ (F(p) - 1) / |grad F| and s = d / (e1^2 |n|),
                // i.e. s = g / (2 e1^2 |grad F|^2) with grad F / 2 = (y0/e0^2, y1/e1^2)
                const double gx = y0 * E.inv_e0sq, gy = y1 * E.inv_e1sq;
                double s = 0.5 * g * E.inv_e1sq / (gx * gx + gy * gy);
                if (!(s > lo && s < hi)) s = 0.5 * (lo + hi);
                for (int it = 0; it < 200; ++it) {
                    // one reciprocal for both factors (s > z1 - 1 > -1 keeps them positive)
                    const double a = s + r0, c = s + 1.0;
                    const double iac = 1.0 / (a * c);
                    const double i0 = c * iac, i1 = a * iac;
                    const double a0 = n0 * i0, a1 = z1 * i1;
                    const double F = a0 * a0 + a1 * a1 - 1.0;
                    if (F > 0.0) lo = s; else if (F < 0.0) hi = s; else break;
                    const double dF = -2.0 * (a0 * a0 * i0 + a1 * a1 * i1);
                    double sn = s - F / dF;
                    const bool newton = sn > lo && sn < hi;
                    if (!newton) sn = 0.5 * (lo + hi);
                    const double step = fabs(sn - s);
                    s = sn;
                    if ((newton && step <= 1e-8 * (1.0 + fabs(s))) || !(hi > lo)) break;
                }
                *c0 = r0 * y0 / (s + r0);
                *c1 = y1 / (s + 1.0);
            } else {
                *c0 = y0;
                *c1 = y1;
            }
        } else {
            *c0 = 0.0;
            *c1 = e1;
        }
    } else {
        const double numer0 = e0 * y0, denom0 = e0 * e0 - e1 * e1;
        if (numer0 < denom0) {
            const double xde0 = numer0 * E.inv_denom0;
            *c0 = e0 * xde0;
            *c1 = e1 * sqrt(1.0 - xde0 * xde0);
        } else {
            *c0 = e0;
            *c1 = 0.0;
        }
    }
}

// Signed distance of (X, Y) to the ellipse (X/a)^2 + (Y/b)^2 = 1 (positive outside) and the
// outward unit normal at the nearest point.
__device__ inline void ellipse_sdf(const EllipseF64& E, double X, double Y, double* sd,
                                   double* nx, double* ny)
{
    const double ax = fabs(X), ay = fabs(Y);
    double cx, cy;
    if (!E.swap) {
        ellipse_nearest_q1(E, ax, ay, &cx, &cy);
    } else {
        ellipse_nearest_q1(E, ay, ax, &cy, &cx);
    }
    cx = X < 0.0 ? -cx : cx;
    cy = Y < 0.0 ? -cy : cy;
    const double dx = X - cx, dy = Y - cy;
    const double dist = sqrt(dx * dx + dy * dy);
    const double level = X * X * E.inv_a2 + Y * Y * E.inv_b2;
    *sd = level < 1.0 ? -dist : dist;
    const double gx = cx * E.inv_a2, gy = cy * E.inv_b2;
    const double ign = 1.0 / sqrt(gx * gx + gy * gy);
    *nx = gx * ign;
    *ny = gy * ign;
}

// Belief of one step, evaluated once: lateral deviation, normal, spread along the normal and the
// barrier value h = max(w_T - nu sigma_y, 0)^2 - e_y^2.
struct BeliefEval {
    double ey, nx, ny, sigma, h;
    double sig_obs[kMaxObstacles];   // spread along each obstacle's gradient direction
};

// Spreads sqrt(a_i^T Sigma a_i) of the half-space constraints from their variances.
__device__ inline void con_sigmas(const ScoreF64& p, const double* cvar, double* sig)
{
#pragma unroll
    for (int i = 0; i < kMaxCon; ++i) sig[i] = i < p.n_con ? sqrt(fmax(cvar[i], 0.0)) : 0.0;
}

// Barrier at mean state x with given spreads: h = min over the constraints (eq. 16) of the track
// walls as eq. 33, each obstacle in the same quadratic form, max(d_i - nu sigma_i, 0)^2 - r_i^2
// with d_i the distance to its centre, and (sig_con non-null) each half-space constraint as the
// heuristic of eq. 13 itself, b_i - a_i^T x - nu sigma_i.
__device__ inline double barrier_at(const ScoreF64& p, const double* x, double ey, double sigma,
                                    const double* sig_obs, const double* sig_con)
{
    const double X = x[0], Y = x[1];
    const double margin = fmax(p.half_width - p.nu * sigma, 0.0);
    double h = margin * margin - ey * ey;
    for (int i = 0; i < p.n_obs; ++i) {
        const double dx = X - p.obs[3 * i], dy = Y - p.obs[3 * i + 1], r = p.obs[3 * i + 2];
        const double m = fmax(sqrt(dx * dx + dy * dy) - p.nu * sig_obs[i], 0.0);
        h = fmin(h, m * m - r * r);
    }
    if (sig_con) {
#pragma unroll
        for (int i = 0; i < kMaxCon; ++i) {
            if (i < p.n_con) {
                const double* a = p.con_a + 6 * i;
                double ax = a[0] * x[0];
#pragma unroll
                for (int j = 1; j < 6; ++j) ax = fma(a[j], x[j], ax);
                h = fmin(h, p.con_b[i] - ax - p.nu * sig_con[i]);
            }
        }
    }
    return h;
}

// sig_con: spreads of the half-space constraints (con_sigmas), or nullptr where the launch
// carries none
__device__ inline BeliefEval eval_belief(const ScoreF64& p, const double* mom,
                                         const double* sig_con = nullptr)
{
    BeliefEval b;
    ellipse_sdf(p.ell, mom[0], mom[1], &b.ey, &b.nx, &b.ny);
    const double var = b.nx * b.nx * mom[6] + 2.0 * b.nx * b.ny * mom[7] + b.ny * b.ny * mom[8];
    b.sigma = sqrt(fmax(var, 0.0));
    for (int i = 0; i < p.n_obs; ++i) {
        // eta = unit vector from the centre to the mean position ((1, 0) at the centre)
        const double dx = mom[0] - p.obs[3 * i], dy = mom[1] - p.obs[3 * i + 1];
        const double d = sqrt(dx * dx + dy * dy);
        const double ex = d > 0.0 ? dx / d : 1.0, ez = d > 0.0 ? dy / d : 0.0;
        const double v = ex * ex * mom[6] + 2.0 * ex * ez * mom[7] + ez * ez * mom[8];
        b.sig_obs[i] = sqrt(fmax(v, 0.0));
    }
    b.h = barrier_at(p, mom, b.ey, b.sigma, b.sig_obs, sig_con);
    return b;
}

// Running cost on the mean (tracking, heading error w.r.t. the counter-clockwise tangent, lateral
// deviation, collision indicator).
__device__ inline double stage_cost(const ScoreF64& p, const double* mom, const BeliefEval& b)
{
    const double tx = -b.ny, ty = b.nx;
    double sp, cp;
    sincos(mom[2], &sp, &cp);
    const double cos_epsi = cp * tx + sp * ty;
    const double dv = mom[3] - p.v_goal;
    double q = p.q_vx * dv * dv + p.q_vy * mom[4] * mom[4] + p.q_r * mom[5] * mom[5] +
               p.q_ey * b.ey * b.ey + p.q_epsi * 2.0 * (1.0 - cos_epsi);
    if (fabs(b.ey) >= p.half_width) q += p.C_obs;
    for (int i = 0; i < p.n_obs; ++i) {
        const double dx = mom[0] - p.obs[3 * i], dy = mom[1] - p.obs[3 * i + 1];
        const double r = p.obs[3 * i + 2];
        if (dx * dx + dy * dy <= r * r) q += p.C_obs;
    }
    return q;
}

// One-step residual of the linear class-kappa condition for a candidate control: the mean is
// pushed through the noise-free model and re-scored with the spreads frozen at step t (sig_con:
// those of the half-space constraints, or nullptr).
__device__ inline double repair_residual(const ScoreF64& p, const double* xbar,
                                         const BeliefEval& be, double h_t, double steer,
                                         double accel, const double* sig_con = nullptr)
{
    double xn[6];
    car_step_f64(p, xbar, steer, accel, xn);
    double ey, nx, ny;
    ellipse_sdf(p.ell, xn[0], xn[1], &ey, &nx, &ny);
    return -barrier_at(p, xn, ey, be.sigma, be.sig_obs, sig_con) + (1.0 - p.gamma) * h_t;
}

}  // namespace bss
