// bss_kernels.hip -- merge, repair-of-the-update and stage kernels of the BSS-MPPI solve for
// gfx950 (MI355X), and the host-side launch shape and launch wrappers.
//
// One solve = two launches on one stream:
//   solve  : (bss_solve.h) rollout, belief moments, scoring and the block's log-sum-exp partial;
//   merge  : one wave per control entry (t, j): rescales the block partials to the global
//            minimum, exp(-(m_b - m)/lambda), and writes v+ = v + N/Z into the other buffer of the
//            ping-pong pair (so no block reads what another writes).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bss_device.h"
#include "bss_internal.h"
#include "bss_wave.h"

namespace bss {

namespace {

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
                                   double& m, double& Z, double& W2, double& nf, double& N,
                                   double& V)
{
    const int lane = (int)(threadIdx.x & 63u);
    const int stride = partial_stride(T);
    // up to four blocks per lane are loaded in one pass (all loads in flight together); larger
    // grids fall back to a second pass over the remaining blocks
    constexpr int kHeld = 4;
    double hm[kHeld], hz[kHeld], hw[kHeld], hn[kHeld], hc[kHeld], hv[kHeld];
#pragma unroll
    for (int i = 0; i < kHeld; ++i) {
        const int b = lane + 64 * i;
        const double* pb = partial + (size_t)(b < G ? b : 0) * stride;
        hm[i] = b < G ? pb[2 * T + 3] : INFINITY;
        hz[i] = b < G ? pb[2 * T] : 0.0;
        hw[i] = b < G ? pb[2 * T + 1] : 0.0;
        hn[i] = b < G ? pb[2 * T + 2] : 0.0;
        hc[i] = b < G ? pb[col] : 0.0;
        hv[i] = b < G ? pb[2 * T + 4] : 0.0;
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
    V = 0.0;
#pragma unroll
    for (int i = 0; i < kHeld; ++i) {
        const double sc = isfinite(hm[i]) ? exp(-(hm[i] - m) / lambda) : 0.0;
        Z += sc * hz[i];
        W2 += sc * sc * hw[i];
        nf += hn[i];
        N += sc * hc[i];
        V += hv[i];
    }
    for (int b = lane + 64 * kHeld; b < G; b += 64) {
        const double* pb = partial + (size_t)b * stride;
        const double mb = pb[2 * T + 3];
        const double sc = isfinite(mb) ? exp(-(mb - m) / lambda) : 0.0;
        Z += sc * pb[2 * T];
        W2 += sc * sc * pb[2 * T + 1];
        nf += pb[2 * T + 2];
        N += sc * pb[col];
        V += pb[2 * T + 4];
    }
    Z = wave_reduce(Z, AddOp());
    W2 = wave_reduce(W2, AddOp());
    nf = wave_reduce(nf, AddOp());
    N = wave_reduce(N, AddOp());
    V = wave_reduce(V, AddOp());
}

__device__ inline void write_stats(double* stats, int col, double vo, bool ok, double m, double Z,
                                   double W2, double nf, double V)
{
    if (col < 2) stats[5 + col] = vo;
    if (col == 0) {
        stats[0] = m;
        stats[1] = Z;
        stats[2] = ok ? Z * Z / W2 : 0.0;
        stats[3] = nf;
        stats[4] = ok ? 0.0 : 5.0;
        stats[7] = V;
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
    double m, Z, W2, nf, N, V;
    merge_entry(d.partial, d.nblocks, T, col, d.sc.lambda, m, Z, W2, nf, N, V);
    if ((threadIdx.x & 63u) == 0) {
        const bool ok = nf > 0.0 && Z > 0.0;
        const double vo = ok ? vi + N / Z : vi;
        d.v[1 - cur][col] = vo;
        write_stats(d.stats, col, vo, ok, m, Z, W2, nf, V);
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
    double m, Z, W2, nf, N, V;
    merge_entry(partial, G, T, col, lambda, m, Z, W2, nf, N, V);
    if ((threadIdx.x & 63u) == 0) {
        const bool ok = nf > 0.0 && Z > 0.0;
        const double vo = ok ? v_in[col] + N / Z : v_in[col];
        v_out[col] = vo;
        write_stats(stats, col, vo, ok, m, Z, W2, nf, V);
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
    block_partial(T, n, S_sh, w_sh, u_sh, v, 0, lambda, 0.0,
                  partial + (size_t)blockIdx.x * partial_stride(T));
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

// Disturbance of a solve through the solve kernel's own path (first two rounds shared per
// particle block and per step, per-block tails, the quad dealing, the lane placement of
// particles): words[k][t][3 ceil(M / 4)][4] of every block and w[k][t][m][3] of every particle.
// One group of L lanes per sample, as in the solve.
template <int P, int L>
__global__ __launch_bounds__(256) void disturbance_kernel(uint32_t key0, uint32_t key1,
                                                          uint32_t s, int K, int M, int T,
                                                          int crn, float* w, uint32_t* words)
{
    const int g = (int)threadIdx.x / L, j = (int)threadIdx.x % L;
    const int k = (int)blockIdx.x * (256 / L) + g;
    if (k >= K) return;   // whole groups leave together (the lane quads stay complete)
    const uint32_t c3w = rng_word3(kTagW, s);
    const uint64_t pk = (uint64_t)kPhiloxM1 * (crn ? 0u : (uint32_t)k);
    const uint32_t hk = (uint32_t)(pk >> 32), lk = (uint32_t)pk;
    constexpr int NB = noise_blocks<P>();
    PhiloxParticle pb[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) pb[i] = philox_particle(noise_block_word<P, L>(j, i), hk, key0, key1);
    const int nblk = 3 * ((M + 3) / 4);
    for (int t = 0; t < T; ++t) {
        const PhiloxStep ps = philox_step((uint32_t)t, c3w, lk, key0, key1);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            uint32_t r0, r1, r2, r3;
            philox10_tail(ps, pb[i], key0, key1, r0, r1, r2, r3);
            const int bw = (int)noise_block_word<P, L>(j, i);
            if (bw < nblk) {
                uint32_t* o = words + (((size_t)k * T + t) * nblk + bw) * 4;
                o[0] = r0;
                o[1] = r1;
                o[2] = r2;
                o[3] = r3;
            }
        }
        NoiseDealer<P> deal{ps, pb, key0, key1, j, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int p = 0; p < P; ++p) {
            float a, b, c;
            deal.next(p, a, b, c);
            const int m = particle_of<P, L>(j, p);
            if (m < M) {
                float* o = w + (((size_t)k * T + t) * M + m) * 3;
                o[0] = a;
                o[1] = b;
                o[2] = c;
            }
        }
    }
}

template <int P>
hipError_t launch_disturbance_p(int lanes, uint32_t key0, uint32_t key1, uint32_t s, int K, int M,
                                int T, int crn, float* w, uint32_t* words, hipStream_t stream)
{
    const dim3 grid((unsigned)((K + 256 / lanes - 1) / (256 / lanes))), block(256);
    switch (lanes) {
    case 8:
        hipLaunchKernelGGL((disturbance_kernel<P, 8>), grid, block, 0, stream, key0, key1, s, K,
                           M, T, crn, w, words);
        break;
    case 16:
        hipLaunchKernelGGL((disturbance_kernel<P, 16>), grid, block, 0, stream, key0, key1, s, K,
                           M, T, crn, w, words);
        break;
    case 32:
        hipLaunchKernelGGL((disturbance_kernel<P, 32>), grid, block, 0, stream, key0, key1, s, K,
                           M, T, crn, w, words);
        break;
    default:
        hipLaunchKernelGGL((disturbance_kernel<P, 64>), grid, block, 0, stream, key0, key1, s, K,
                           M, T, crn, w, words);
        break;
    }
    return hipGetLastError();
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

size_t solve_base_lds_bytes(int lanes, int T, int ppl, bool split, bool resample)
{
    const int groups = 256 / lanes;
    return (size_t)2 * groups * sizeof(double) + (size_t)groups * T * sizeof(float2) +
           (split ? (size_t)2 * ppl * (resample ? 9 : 3) * 256 * sizeof(float) : 0);
}

size_t solve_lds_bytes(int lanes, int T, int ppl, bool split, bool resample, bool con)
{
    const int groups = 256 / lanes;
    return solve_base_lds_bytes(lanes, T, ppl, split, resample) +
           (size_t)(split ? 2 : 1) * groups * moment_region_doubles(lanes, con) * sizeof(double);
}

bool split_fits(int lanes, int T, int ppl, bool resample, bool con, size_t static_lds)
{
    return solve_lds_bytes(lanes, T, ppl, true, resample, con) + static_lds <= kMaxLdsPerBlock;
}

size_t solve8_lds_bytes(int lanes, int T)
{
    const int groups = 256 / lanes;
    return (size_t)2 * groups * sizeof(double) + (size_t)groups * T * sizeof(float2);
}

size_t record_lds_bytes(int lanes, int T, int n_con)
{
    return (size_t)(256 / lanes) * (T + 1) * (9 + n_con) * sizeof(double);
}

bool split_pays(int nblocks, int lanes, int T, int ppl)
{
    // fewer than two waves per SIMD (256 CUs x 4 SIMDs, four waves per block), and room for the
    // noise ring
    return (int64_t)nblocks * 4 < 2 * 1024 && solve_base_lds_bytes(lanes, T, ppl, true) <= kMaxLds;
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
        // default: about four particles per lane, 16..64 lanes per sample; a launch with fewer
        // sample lanes than one wave per SIMD (K L < 64 x 1024) is latency-bound, so its
        // particles are spread over more lanes, fewer per lane, until it has a wave per SIMD or
        // one particle per lane (measured: 8-state vehicle K=1000, M=20: 0.19 -> 0.11 ms;
        // K=512, M=64: 0.109 -> 0.076 ms; re-sampling K=1024: 0.280 -> 0.202 ms)
        int lanes = 16;
        while (lanes < 64 && lanes * 4 < M) lanes <<= 1;
        while (lanes < 64 && ppl_for(M, lanes) > 1 && (int64_t)K * lanes < 64 * 1024) lanes <<= 1;
        s.lanes = lanes;
    }
    s.ppl = ppl_for(M, s.lanes);
    while ((s.ppl > 8 || solve_base_lds_bytes(s.lanes, T, s.ppl, false) > kMaxLds) &&
           s.lanes < 64) {
        s.lanes <<= 1;
        s.ppl = ppl_for(M, s.lanes);
    }
    const bool fits = solve_base_lds_bytes(s.lanes, T, s.ppl, true) <= kMaxLds;
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
                        hipStream_t stream, uint32_t* queue)
{
    if (nblocks <= 0) return hipSuccess;
    split = split && !shield && !(resample && con);
    switch (ppl) {
    case 0:
        return launch_solve_pm(inst, blocks, nblocks, shield, split, resample, con,
                               lds, x0_base, Sigma0_base, extra_shift, queue, stream);
    case 1:
        return launch_solve_p1(inst, blocks, nblocks, shield, split, resample, con,
                                    lds, x0_base, Sigma0_base, extra_shift, queue, stream);
    case 2:
        return launch_solve_p2(inst, blocks, nblocks, shield, split, resample, con,
                                    lds, x0_base, Sigma0_base, extra_shift, queue, stream);
    case 4:
        return launch_solve_p4(inst, blocks, nblocks, shield, split, resample, con,
                                    lds, x0_base, Sigma0_base, extra_shift, queue, stream);
    case 8:
        return launch_solve_p8(inst, blocks, nblocks, shield, split, resample, con,
                                    lds, x0_base, Sigma0_base, extra_shift, queue, stream);
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

hipError_t launch_disturbance(int lanes, int ppl, uint32_t key0, uint32_t key1, uint32_t s,
                              int K, int M, int T, int crn, float* w, uint32_t* words,
                              hipStream_t stream)
{
    if (K <= 0 || T <= 0 || M <= 0) return hipSuccess;
    switch (ppl) {
    case 1: return launch_disturbance_p<1>(lanes, key0, key1, s, K, M, T, crn, w, words, stream);
    case 2: return launch_disturbance_p<2>(lanes, key0, key1, s, K, M, T, crn, w, words, stream);
    case 4: return launch_disturbance_p<4>(lanes, key0, key1, s, K, M, T, crn, w, words, stream);
    case 8: return launch_disturbance_p<8>(lanes, key0, key1, s, K, M, T, crn, w, words, stream);
    default: return hipErrorInvalidValue;
    }
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
