// bss_kernels.hip -- HIP kernels of the BSS-MPPI solve for gfx950 (MI355X).
//
// One solve = three launches on one stream:
//   rollout  : L lanes per control sample k (256/L samples per 256-thread block), P particles per
//              lane in registers.  Draws eps_{k,t} (Philox tag 0) lane-parallel over t, optionally
//              shield-repairs u_{k,t} per step, propagates the M particles with the single-
//              precision midpoint rule plus the disturbance (tag 1), and reduces the particle
//              mean and position covariance across the L lanes in double precision every step.
//   score    : one wave per sample, lanes parallel over t: signed distance, sigma_y, barrier h,
//              running/terminal cost, control cost, C_safe on the transitions; S_k in double.
//   update   : log-sum-exp K-reduction in double precision: each block takes a slice of the
//              samples, forms weights relative to its own minimum cost, and the last block to
//              finish merges the slices with the rescaling exp(-(m_b - m)/lambda), then writes
//              v+ = v + N/Z in place.
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

template <int L>
__device__ __forceinline__ double group_sum(double x)
{
#pragma unroll
    for (int mask = 1; mask < L; mask <<= 1) x += __shfl_xor(x, mask, L);
    return x;
}

// ----------------------------------------------------------------------------------------------
// rollout
// ----------------------------------------------------------------------------------------------
template <int L, int P, bool SHIELD>
__global__ __launch_bounds__(256) void rollout_kernel(SolveArgs a)
{
    constexpr int kGroups = 256 / L;
    extern __shared__ float2 u_sh[];
    const int T = a.T, M = a.M;
    const int g = threadIdx.x / L;
    const int j = threadIdx.x % L;
    const int k = blockIdx.x * kGroups + g;
    const bool active = k < a.K;
    float2* us = u_sh + g * T;
    const uint32_t s = a.solve_index;

    // ---- phase 1: control samples u_{k,t} = clip(v_t + eps_{k,t}), lane-parallel over t ----
    if (active) {
        for (int t = j; t < T; t += L) {
            uint32_t c0 = (uint32_t)t, c1 = 0u, c2 = (uint32_t)k, c3 = rng_word3(kTagEps, s);
            philox10(c0, c1, c2, c3, a.key0, a.key1);
            float z0, z1;
            bm_pair(c0, c1, z0, z1);
            const float v0 = (float)a.v[2 * t], v1 = (float)a.v[2 * t + 1];
            const float u0 = fminf(fmaxf(fmaf(a.sig_eps0, z0, v0), -a.steer_max), a.steer_max);
            const float u1 = fminf(fmaxf(fmaf(a.sig_eps1, z1, v1), -a.accel_max), a.accel_max);
            us[t] = make_float2(u0, u1);
            if (!SHIELD) {
                float2* uo = reinterpret_cast<float2*>(a.u) + (size_t)k * T + t;
                *uo = make_float2(u0, u1);
            }
        }
    }
    __syncthreads();
    if (!active) return;

    // ---- phase 2: particles ----
    double x0[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) x0[i] = a.x0[i];
    const bool spread = a.Sigma0 != nullptr;
    double L0[36];
    if (spread) chol6(a.Sigma0, L0);

    // state relative to the estimate: position and heading as compensated (sum, correction)
    float Xs[P], Xc[P], Ys[P], Yc[P], Ps[P], Pc[P], vx[P], vy[P], vr[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int m = j + p * L;
        double dev[6] = {0, 0, 0, 0, 0, 0};
        if (spread) {
            double xi[6];
#pragma unroll
            for (int blk = 0; blk < 2; ++blk) {
                uint32_t c0 = (uint32_t)blk, c1 = (uint32_t)m, c2 = (uint32_t)k,
                         c3 = rng_word3(kTagInit, s);
                philox10(c0, c1, c2, c3, a.key0, a.key1);
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
    const double rev0d = x0[2] * 0.15915494309189535;
    const float rev0 = (float)(rev0d - rint(rev0d));
    const CarF32 car = a.car;

    double* mom_k = a.mom + (size_t)k * (T + 1) * 9;
    // belief at t = 0 is the given estimate
    double bel[9];
#pragma unroll
    for (int i = 0; i < 6; ++i) bel[i] = x0[i];
    bel[6] = spread ? a.Sigma0[0] : 0.0;
    bel[7] = spread ? a.Sigma0[1] : 0.0;
    bel[8] = spread ? a.Sigma0[7] : 0.0;
    if (j == 0) {
#pragma unroll
        for (int i = 0; i < 9; ++i) mom_k[i] = bel[i];
    }
    const uint32_t c3w = rng_word3(kTagW, s);
    const double invM = 1.0 / (double)M;
    const double invM1 = M > 1 ? 1.0 / (double)(M - 1) : 0.0;

    for (int t = 0; t < T; ++t) {
        float2 uu = us[t];
        if (SHIELD) {
            const ScoreF64& sc = a.sc;
            if (sc.shield_iters > 0) {
                const BeliefEval be = eval_belief(sc, bel);
                const double margin = fmax(sc.half_width - sc.nu * be.sigma, 0.0);
                const double margin2 = margin * margin;
                const double fd = sc.shield_fd;
                const int role = j < 5 ? j : 0;
                const double o0 = role == 1 ? fd : (role == 2 ? -fd : 0.0);
                const double o1 = role == 3 ? fd : (role == 4 ? -fd : 0.0);
                double us0 = uu.x, us1 = uu.y;
                for (int it = 0; it < sc.shield_iters; ++it) {
                    // lanes 0-4 of the group evaluate r at u and at the four difference points
                    const double rv = repair_residual(sc, bel, margin2, be.h, us0 + o0, us1 + o1);
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
                float2* uo = reinterpret_cast<float2*>(a.u) + (size_t)k * T + t;
                *uo = uu;
            }
        }
        const StepF32 st = make_step(car, uu.x, uu.y);
        double sX = 0, sY = 0, sP = 0, svx = 0, svy = 0, svr = 0, sXX = 0, sXY = 0, sYY = 0;
        double refX = 0.0, refY = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int m = j + p * L;
            uint32_t c0 = (uint32_t)t, c1 = (uint32_t)m, c2 = (uint32_t)k, c3 = c3w;
            philox10(c0, c1, c2, c3, a.key0, a.key1);
            float w0, w1;
            bm_pair(c0, c1, w0, w1);
            const float w2 = bm_cos(c2, c3);

            float dX1, dY1, dvx1, dvy1, dr1;
            car_field_f32(car, st, fmaf(Ps[p], kInv2Pi, rev0), vx[p], vy[p], vr[p], dX1, dY1,
                          dvx1, dvy1, dr1);
            const float pm = fmaf(car.half_dt, vr[p], Ps[p]);
            const float vxm = fmaf(car.half_dt, dvx1, vx[p]);
            const float vym = fmaf(car.half_dt, dvy1, vy[p]);
            const float vrm = fmaf(car.half_dt, dr1, vr[p]);
            float dX2, dY2, dvx2, dvy2, dr2;
            car_field_f32(car, st, fmaf(pm, kInv2Pi, rev0), vxm, vym, vrm, dX2, dY2, dvx2, dvy2,
                          dr2);
            kahan_add(Xs[p], Xc[p], car.dt * dX2);
            kahan_add(Ys[p], Yc[p], car.dt * dY2);
            kahan_add(Ps[p], Pc[p], car.dt * vrm);
            vx[p] = fmaf(a.sig_w0, w0, fmaf(car.dt, dvx2, vx[p]));
            vy[p] = fmaf(a.sig_w1, w1, fmaf(car.dt, dvy2, vy[p]));
            vr[p] = fmaf(a.sig_w2, w2, fmaf(car.dt, dr2, vr[p]));

            if (p == 0) {
                // shift for the covariance sums: particle 0 of the sample (lane 0 of the group)
                refX = (double)__shfl(Xs[0], 0, L) - (double)__shfl(Xc[0], 0, L);
                refY = (double)__shfl(Ys[0], 0, L) - (double)__shfl(Yc[0], 0, L);
            }
            if (m < M) {   // masked particles beyond M contribute nothing
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
            }
        }
        sX = group_sum<L>(sX);
        sY = group_sum<L>(sY);
        sP = group_sum<L>(sP);
        svx = group_sum<L>(svx);
        svy = group_sum<L>(svy);
        svr = group_sum<L>(svr);
        sXX = group_sum<L>(sXX);
        sXY = group_sum<L>(sXY);
        sYY = group_sum<L>(sYY);
        // moments: sums of positions shifted by particle 0, heading relative to the estimate
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
        if (j == 0) {
            double* rec = mom_k + (size_t)(t + 1) * 9;
#pragma unroll
            for (int i = 0; i < 9; ++i) rec[i] = bel[i];
        }
    }
}

// ----------------------------------------------------------------------------------------------
// score: one wave per sample
// ----------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void score_kernel(int K, int T, ScoreF64 sc, const double* mom,
                                                    const float* u, const double* v, double* S)
{
    extern __shared__ double h_sh[];   // [4][T+1]
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int k = blockIdx.x * 4 + w;
    const bool active = k < K;
    double* hs = h_sh + w * (T + 1);
    double part = 0.0;
    if (active) {
        const double* mk = mom + (size_t)k * (T + 1) * 9;
        for (int t = lane; t <= T; t += 64) {
            const double* rec = mk + (size_t)t * 9;
            const BeliefEval be = eval_belief(sc, rec);
            double q = stage_cost(sc, rec, be);
            if (t == T) {
                q *= sc.phi_scale;
            } else {
                const float2 ut = reinterpret_cast<const float2*>(u)[(size_t)k * T + t];
                q += sc.gamma_u * (v[2 * t] * sc.inv_var0 * (double)ut.x +
                                   v[2 * t + 1] * sc.inv_var1 * (double)ut.y);
            }
            hs[t] = be.h;
            part += q;
        }
    }
    __syncthreads();
    if (!active) return;
    for (int t = lane; t <= T; t += 64) {
        if (t >= 1) {
            const double viol = -hs[t] + (1.0 - sc.gamma) * hs[t - 1];
            part += sc.C_cbf * fmax(viol, 0.0);
        }
    }
#pragma unroll
    for (int mask = 1; mask < 64; mask <<= 1) part += __shfl_xor(part, mask, 64);
    if (lane == 0) S[k] = part;
}

// ----------------------------------------------------------------------------------------------
// update: log-sum-exp K-reduction with the weighted perturbation average
// ----------------------------------------------------------------------------------------------
constexpr int kUpdateSlice = 256;   // samples per block

__device__ __forceinline__ double block_min_256(double x, double* red)
{
    const int tid = threadIdx.x;
    red[tid] = x;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) red[tid] = fmin(red[tid], red[tid + off]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_sum_256(double x, double* red)
{
    const int tid = threadIdx.x;
    red[tid] = x;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) red[tid] += red[tid + off];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void update_kernel(UpdateArgs a)
{
    __shared__ double w_sh[kUpdateSlice];
    __shared__ double red[256];
    __shared__ bool is_last;
    const int tid = threadIdx.x;
    const int K = a.K, T = a.T;
    const int k_begin = blockIdx.x * kUpdateSlice;
    const int k_end = min(K, k_begin + kUpdateSlice);
    const int nk = k_end - k_begin;
    const int width = 2 * T + 3;   // numerators, Z, sum w^2, finite count
    double* part = a.partial + (size_t)blockIdx.x * (width + 1);

    // block-local minimum over finite costs
    double Sk = INFINITY;
    bool fin = false;
    if (tid < nk) {
        Sk = a.S[k_begin + tid];
        fin = isfinite(Sk);
    }
    const double mb = block_min_256(fin ? Sk : INFINITY, red);
    const double wk = (fin && isfinite(mb)) ? exp(-(Sk - mb) / a.lambda) : 0.0;
    if (tid < nk) w_sh[tid] = wk;
    const double Zb = block_sum_256(wk, red);
    const double W2b = block_sum_256(wk * wk, red);
    const double nf = block_sum_256(fin ? 1.0 : 0.0, red);
    for (int i = tid; i < 2 * T; i += 256) {
        const double vi = a.v[i];
        double acc = 0.0;
        for (int q = 0; q < nk; ++q) {
            const double w = w_sh[q];
            const double ui = (double)a.u[(size_t)(k_begin + q) * 2 * T + i];
            acc += w * (ui - vi);
        }
        part[i] = acc;
    }
    if (tid == 0) {
        part[2 * T] = Zb;
        part[2 * T + 1] = W2b;
        part[2 * T + 2] = nf;
        part[2 * T + 3] = mb;
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        const uint32_t done = atomicAdd(a.counter, 1u);
        is_last = (done == (uint32_t)(gridDim.x - 1));
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();

    // last block: merge the slices in a fixed order
    const int G = gridDim.x;
    double m = INFINITY;
    for (int b = 0; b < G; ++b) m = fmin(m, a.partial[(size_t)b * (width + 1) + 2 * T + 3]);
    double Z = 0.0, W2 = 0.0, n_fin = 0.0;
    for (int b = 0; b < G; ++b) {
        const double* pb = a.partial + (size_t)b * (width + 1);
        const double sc = isfinite(pb[2 * T + 3]) ? exp(-(pb[2 * T + 3] - m) / a.lambda) : 0.0;
        Z += sc * pb[2 * T];
        W2 += sc * sc * pb[2 * T + 1];
        n_fin += pb[2 * T + 2];
    }
    const bool ok = n_fin > 0.0 && Z > 0.0;
    for (int i = tid; i < 2 * T; i += 256) {
        double num = 0.0;
        for (int b = 0; b < G; ++b) {
            const double* pb = a.partial + (size_t)b * (width + 1);
            const double sc = isfinite(pb[2 * T + 3]) ? exp(-(pb[2 * T + 3] - m) / a.lambda) : 0.0;
            num += sc * pb[i];
        }
        if (ok) a.v[i] = a.v[i] + num / Z;
    }
    __syncthreads();
    if (tid == 0) {
        a.stats[0] = m;
        a.stats[1] = Z;
        a.stats[2] = ok ? Z * Z / W2 : 0.0;
        a.stats[3] = n_fin;
        a.stats[4] = ok ? 0.0 : 5.0;
        a.stats[5] = a.v[0];
        a.stats[6] = a.v[1];
        a.stats[7] = 0.0;
        *a.counter = 0u;
    }
}

__global__ void shift_kernel(double* v, int T)
{
    // one block: read everything, then write shifted
    const int tid = threadIdx.x;
    double a0 = 0.0, a1 = 0.0;
    for (int base = 0; base < T; base += 256) {
        const int t = base + tid;
        const bool ok = t < T;
        const int src = (t + 1 < T) ? t + 1 : T - 1;
        if (ok) {
            a0 = v[2 * src];
            a1 = v[2 * src + 1];
        }
        __syncthreads();
        if (ok) {
            v[2 * t] = a0;
            v[2 * t + 1] = a1;
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------------------------
// stand-alone kernels for staged checks
// ----------------------------------------------------------------------------------------------
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

__global__ void sdf_kernel(double a, double b, const double* pts, double* out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double sd, nx, ny;
    ellipse_sdf(a, b, pts[2 * i], pts[2 * i + 1], &sd, &nx, &ny);
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
        const double margin = fmax(sc.half_width - sc.nu * be.sigma, 0.0);
        const double margin2 = margin * margin;
        const double fd = sc.shield_fd;
        for (int it = 0; it < sc.shield_iters; ++it) {
            const double r0 = repair_residual(sc, bel, margin2, be.h, us0, us1);
            if (!(r0 > 0.0)) break;
            const double g0 = (repair_residual(sc, bel, margin2, be.h, us0 + fd, us1) -
                               repair_residual(sc, bel, margin2, be.h, us0 - fd, us1)) / (2.0 * fd);
            const double g1 = (repair_residual(sc, bel, margin2, be.h, us0, us1 + fd) -
                               repair_residual(sc, bel, margin2, be.h, us0, us1 - fd)) / (2.0 * fd);
            const double den = g0 * g0 + g1 * g1 + sc.shield_gmin * sc.shield_gmin;
            us0 = clampd(us0 - r0 * g0 / den, -sc.steer_max, sc.steer_max);
            us1 = clampd(us1 - r0 * g1 / den, -sc.accel_max, sc.accel_max);
        }
    }
    u_out[2 * i] = us0;
    u_out[2 * i + 1] = us1;
}

template <int L, int P>
hipError_t launch_rollout_lp(const SolveArgs& a, bool shield, hipStream_t stream)
{
    constexpr int kGroups = 256 / L;
    const unsigned blocks = (unsigned)((a.K + kGroups - 1) / kGroups);
    const size_t lds = (size_t)kGroups * a.T * sizeof(float2);
    if (shield)
        hipLaunchKernelGGL((rollout_kernel<L, P, true>), dim3(blocks), dim3(256), lds, stream, a);
    else
        hipLaunchKernelGGL((rollout_kernel<L, P, false>), dim3(blocks), dim3(256), lds, stream, a);
    return hipGetLastError();
}

template <int L>
hipError_t launch_rollout_l(const SolveArgs& a, int ppl, bool shield, hipStream_t stream)
{
    switch (ppl) {
    case 1: return launch_rollout_lp<L, 1>(a, shield, stream);
    case 2: return launch_rollout_lp<L, 2>(a, shield, stream);
    case 4: return launch_rollout_lp<L, 4>(a, shield, stream);
    case 8: return launch_rollout_lp<L, 8>(a, shield, stream);
    default: return hipErrorInvalidValue;
    }
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

LaunchShape choose_shape(int K, int M, int T, int requested_lanes)
{
    (void)K;
    (void)T;
    LaunchShape s;
    if (requested_lanes == 8 || requested_lanes == 16 || requested_lanes == 32 ||
        requested_lanes == 64) {
        s.lanes = requested_lanes;
    } else {
        // default: about four particles per lane, 8..64 lanes per sample
        int lanes = 8;
        while (lanes < 64 && lanes * 4 < M) lanes <<= 1;
        s.lanes = lanes;
    }
    s.ppl = ppl_for(M, s.lanes);
    while (s.ppl > 8 && s.lanes < 64) {
        s.lanes <<= 1;
        s.ppl = ppl_for(M, s.lanes);
    }
    return s;
}

hipError_t launch_rollout(const SolveArgs& a, LaunchShape shape, hipStream_t stream)
{
    const bool shield = a.sc.shield_iters > 0;
    switch (shape.lanes) {
    case 8: return launch_rollout_l<8>(a, shape.ppl, shield, stream);
    case 16: return launch_rollout_l<16>(a, shape.ppl, shield, stream);
    case 32: return launch_rollout_l<32>(a, shape.ppl, shield, stream);
    case 64: return launch_rollout_l<64>(a, shape.ppl, shield, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_score(const SolveArgs& a, hipStream_t stream)
{
    const unsigned blocks = blocks_for(a.K, 4);
    const size_t lds = (size_t)4 * (a.T + 1) * sizeof(double);
    hipLaunchKernelGGL(score_kernel, dim3(blocks), dim3(256), lds, stream, a.K, a.T, a.sc, a.mom,
                       a.u, a.v, a.S);
    return hipGetLastError();
}

int update_groups(int K) { return (K + kUpdateSlice - 1) / kUpdateSlice; }

hipError_t launch_update(const UpdateArgs& a, hipStream_t stream)
{
    hipLaunchKernelGGL(update_kernel, dim3(a.groups), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_shift(double* v, int T, hipStream_t stream)
{
    hipLaunchKernelGGL(shift_kernel, dim3(1), dim3(256), 0, stream, v, T);
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
    hipLaunchKernelGGL(sdf_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, stream, a, b, pts, out,
                       n);
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
