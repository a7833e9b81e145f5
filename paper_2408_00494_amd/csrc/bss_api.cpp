// bss_api.cpp -- C ABI of libbssmppi: parameter checks, contexts, device buffers and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <cstddef>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/bssmppi.h"
#include "bss_host.h"
#include "bss_internal.h"

using namespace bss;

namespace bss {

namespace {
thread_local std::string g_err;
}  // namespace

const char* last_error_message() { return g_err.c_str(); }

bss_status fail(bss_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

bss_status device_fail(hipError_t e, const char* what)
{
    return fail(BSS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }
bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Upper-tail normal quantile: the x with erfc(x / sqrt 2) / 2 = delta, by Newton's method from
// x = 0 (the tail is convex and decreasing for x > 0, so the iterates increase monotonically).
double gaussian_backoff(double delta)
{
    const double inv_sqrt2 = 0.70710678118654752440;
    const double inv_sqrt2pi = 0.39894228040143267794;
    double x = 0.0;
    if (delta >= 0.5) return 0.0;
    for (int it = 0; it < 200; ++it) {
        const double f = 0.5 * std::erfc(x * inv_sqrt2) - delta;
        const double df = -inv_sqrt2pi * std::exp(-0.5 * x * x);
        const double xn = x - f / df;
        if (std::fabs(xn - x) <= 1e-15 * std::fabs(xn)) {
            x = xn;
            break;
        }
        x = xn;
    }
    return x;
}

double backoff_of(const bss_params& p)
{
    if (p.backoff == 1) return std::sqrt((1.0 - p.delta) / p.delta);
    return gaussian_backoff(p.delta);
}

ScoreF64 make_score(const bss_params& p)
{
    ScoreF64 s;
    s.m = p.m;
    s.Iz = p.Iz;
    s.lf = p.lf;
    s.lr = p.lr;
    s.Cf = p.Cf;
    s.Cr = p.Cr;
    s.mu = p.mu;
    s.g = p.g;
    s.v_min = p.v_min;
    s.dt = p.dt;
    s.steer_max = p.steer_max;
    s.accel_max = p.accel_max;
    s.inv_var0 = p.sigma_eps[0] > 0.0 ? 1.0 / (p.sigma_eps[0] * p.sigma_eps[0]) : 0.0;
    s.inv_var1 = p.sigma_eps[1] > 0.0 ? 1.0 / (p.sigma_eps[1] * p.sigma_eps[1]) : 0.0;
    s.gamma_u = p.gamma_u;
    s.v_goal = p.v_goal;
    s.q_vx = p.q_vx;
    s.q_vy = p.q_vy;
    s.q_r = p.q_r;
    s.q_ey = p.q_ey;
    s.q_epsi = p.q_epsi;
    s.C_cbf = p.C_cbf;
    s.C_obs = p.C_obs;
    s.phi_scale = p.phi_scale;
    s.ell_a = p.ell_a;
    s.ell_b = p.ell_b;
    s.half_width = p.half_width;
    s.ell = make_ellipse(p.ell_a, p.ell_b);
    s.nu = backoff_of(p);
    s.gamma = p.gamma;
    s.lambda = p.lambda;
    s.shield_iters = p.shield_iters;
    s.shield_gmin = p.shield_gmin;
    s.shield_fd = p.shield_fd;
    s.n_obs = p.n_obs;
    for (int i = 0; i < 3 * kMaxObstacles; ++i) s.obs[i] = p.obs[i];
    s.n_con = p.n_con;
    for (int i = 0; i < 6 * kMaxCon; ++i) s.con_a[i] = p.con_a[i];
    for (int i = 0; i < kMaxCon; ++i) s.con_b[i] = p.con_b[i];
    const double L = p.lf + p.lr;
    s.Ffm = p.mu * p.m * p.g * p.lr / L;
    s.Frm = p.mu * p.m * p.g * p.lf / L;
    s.inv_m = 1.0 / p.m;
    s.inv_Iz = 1.0 / p.Iz;
    return s;
}

CarF32 make_car(const bss_params& p)
{
    CarF32 c;
    const double L = p.lf + p.lr;
    c.dt = (float)p.dt;
    c.half_dt = (float)(0.5 * p.dt);
    c.lf = (float)p.lf;
    c.lr = (float)p.lr;
    c.cf_m = (float)(p.Cf / p.m);
    c.cr_m = (float)(p.Cr / p.m);
    c.fF_max = (float)(p.mu * p.g * p.lr / L);
    c.fR_max = (float)(p.mu * p.g * p.lf / L);
    c.m_Iz = (float)(p.m / p.Iz);
    c.v_min = (float)p.v_min;
    return c;
}

Car8F32 make_car8(const bss_params& p)
{
    Car8F32 c;
    const int n = p.n_sub > 0 ? p.n_sub : 1;
    const double L = p.lf + p.lr;
    const double Fzf = p.m * p.g * p.lr / L, Fzr = p.m * p.g * p.lf / L;
    c.h = (float)(p.dt / n);
    c.half_h = (float)(0.5 * p.dt / n);
    c.n_sub = n;
    c.lf = (float)p.lf;
    c.lr = (float)p.lr;
    c.inv_m = (float)(1.0 / p.m);
    c.inv_Iz = (float)(1.0 / p.Iz);
    c.Rw = (float)p.Rw;
    c.Rw_Iw = (float)(p.Rw / p.Iw);
    c.Tmax_Iw = (float)(p.T_max / p.Iw);
    c.muFzf = (float)(p.mu * Fzf);
    c.muFzr = (float)(p.mu * Fzr);
    const double ff = p.mu * p.pac_D * Fzf, fr = p.mu * p.pac_D * Fzr;
    c.inv_fmaxf = ff > 0.0 ? (float)(1.0 / ff) : 0.0f;
    c.inv_fmaxr = fr > 0.0 ? (float)(1.0 / fr) : 0.0f;
    c.B = (float)p.pac_B;
    c.C = (float)p.pac_C;
    c.D = (float)p.pac_D;
    c.E = (float)p.pac_E;
    c.v_min = (float)p.v_min;
    c.kappa0 = (float)(2.0 * M_PI / p.track_len);
    c.kappa_amp = (float)p.kappa_amp;
    c.s_rev = (float)(2.0 / p.track_len);
    return c;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

InstanceDesc make_desc(const bss_params& p)
{
    InstanceDesc d{};
    d.K = p.K;
    d.M = p.M;
    d.T = p.T;
    d.key0 = (uint32_t)p.seed;
    d.key1 = (uint32_t)(p.seed >> 32);
    d.steer_max = (float)p.steer_max;
    d.accel_max = (float)p.accel_max;
    d.sig_eps0 = (float)p.sigma_eps[0];
    d.sig_eps1 = (float)p.sigma_eps[1];
    d.sig_w0 = (float)p.sigma_w[0];
    d.sig_w1 = (float)p.sigma_w[1];
    d.sig_w2 = (float)p.sigma_w[2];
    d.belief = p.belief;
    d.crn = p.crn;
    d.sig_w_speed = (float)p.sigma_w_speed;
    d.vehicle = p.vehicle;
    d.car = make_car(p);
    d.car8 = make_car8(p);
    d.sc = make_score(p);
    return d;
}

bool samples_shielded(const bss_params& p) { return p.shield_iters > 0 && p.local_repair != 2; }
bool launch_shield(const bss_params& p) { return samples_shielded(p); }
bool launch_resample(const bss_params& p) { return p.belief != 0; }
bool shape_for_shield(const bss_params& p)
{
    return samples_shielded(p) && p.belief == 0 && p.n_con == 0;
}

void append_blocks(std::vector<BlockDesc>& out, int inst, int K, int lanes)
{
    const int groups = 256 / lanes;
    for (int k0 = 0; k0 < K; k0 += groups) out.push_back(BlockDesc{inst, k0});
}

}  // namespace bss

struct bss_ctx {
    bss_params p;
    bss_allocator alloc;
    bool has_alloc;
    hipStream_t stream;
    void* block;              // one device allocation holding every buffer below
    InstanceDesc desc;        // host copy of the static descriptor fields
    InstanceDesc* d_desc;     // device descriptor (state fields advanced on the device)
    BlockDesc* d_blocks;      // solve grid of this context
    MergeDesc* d_cols;        // merge grid of this context
    double* x0;               // staging [6]
    double* Sigma0;           // staging [36]
    double* host;             // pinned [64]
    LaunchShape shape;
    size_t lds;
    int pending_shift;        // warm-start shifts requested on the host since the last solve
    int32_t outputs;
    bool timing;
    std::vector<hipEvent_t> ev;   // pairs (start, stop)
    size_t ev_used;
    bss_batch* batch;         // batch that currently owns the context, or nullptr
    int batch_index;          // index of the context in that batch
    // repair of the updated sequence (local_repair != 0): its descriptor (host copy and device),
    // one-block grid, its own launch shape and the LDS of that launch
    InstanceDesc rdesc;
    InstanceDesc* d_rdesc;
    BlockDesc* d_rblock;
    LaunchShape rshape;
    size_t rlds;
};

struct bss_batch {
    std::vector<bss_ctx*> ctxs;
    int n;
    hipStream_t stream;
    void* block;
    InstanceDesc* d_desc;     // [n]
    InstanceDesc* d_backup;   // [n] (autotuning)
    BlockDesc* d_blocks;
    MergeDesc* d_cols;
    double* d_x0;             // [n][6]
    uint32_t* d_queue;        // work-queue counter of the persistent grid
    int nblocks, ncols, shift_after;
    int ppl;                  // particles per lane of every member, 0: each member's own
    std::vector<int> member_ppl;  // each member's particles per lane when ppl == 0
    bool persistent;          // solve grid: resident blocks taking the block table from a queue
    bool split;               // 512-thread blocks with noise-producing waves
    bool resample;            // some member redraws its particles every step
    bool con;                 // some member has half-space constraints
    std::vector<int> lanes;   // lanes per sample of each member in the current layout
    std::vector<int> ppls;    // particles per lane of each member in the current layout
    size_t lds;
    bool shield;
    hipGraph_t graph;
    hipGraphExec_t exec;
    bool captured;
};

namespace {

constexpr size_t kStateOffset = offsetof(InstanceDesc, cur);
constexpr size_t kStateBytes = offsetof(InstanceDesc, shift_after) - offsetof(InstanceDesc, cur);

size_t max_blocks(int K) { return (size_t)solve_blocks(K, 64); }

// sizes, params and launch shape of a context's descriptor (state fields zero, buffers unset);
// its repair iterations are those of the sampled controls (none when only the update is repaired)
void fill_desc(bss_ctx* c)
{
    c->desc = make_desc(c->p);
    c->desc.lanes = c->shape.lanes;
    c->desc.ppl = c->shape.ppl;
    c->desc.nblocks = solve_blocks(c->p.K, c->shape.lanes);
    if (!samples_shielded(c->p)) c->desc.sc.shield_iters = 0;
}

std::vector<BlockDesc> block_table(int inst, int K, int lanes)
{
    std::vector<BlockDesc> out;
    append_blocks(out, inst, K, lanes);
    return out;
}

// Static LDS beside a solve block's dynamic LDS: the variants with the re-sampling compiled in
// hold its 32 KB of sums (the generic constraint variant too), every variant a few block slots.
static size_t static_lds_margin(const bss_params& p)
{
    const bool rs_compiled = launch_resample(p) || (p.n_con > 0 && launch_shield(p));
    return (rs_compiled ? kResampleStaticLds : 0) + kStaticLdsSlots;
}

// Belief records on chip (rec_lds) when no output asks for them and their LDS costs no residency:
// the blocks the grid needs per CU must still fit next to each other.
bool records_on_chip(const bss_ctx* c, size_t base_lds)
{
    if ((c->outputs & BSS_OUT_BELIEFS) || c->p.vehicle != 0) return false;
    const size_t per_block = base_lds + record_lds_bytes(c->shape.lanes, c->p.T, c->p.n_con) +
                             static_lds_margin(c->p);
    if (per_block > kMaxLdsPerBlock) return false;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return false;
    const int64_t per_cu_needed = (solve_blocks(c->p.K, c->shape.lanes) + cus - 1) / cus;
    return (int64_t)(kMaxLdsPerBlock / per_block) >= per_cu_needed;
}

hipError_t upload_shape(bss_ctx* c)
{
    c->desc.lanes = c->shape.lanes;
    c->desc.ppl = c->shape.ppl;
    c->desc.nblocks = solve_blocks(c->p.K, c->shape.lanes);
    // the noise split: not with the repair of the samples nor the generic constraint variant; with
    // the re-sampling draw the noise waves also draw its normals, in a ring three times as large,
    // which must fit beside the kernel's static LDS
    const bool rs = launch_resample(c->p);
    c->shape.split = c->shape.split && !launch_shield(c->p) && c->p.vehicle == 0 &&
                     !(rs && c->p.n_con > 0) &&
                     split_fits(c->shape.lanes, c->p.T, c->shape.ppl, rs, c->p.n_con > 0,
                                static_lds_margin(c->p));
    c->lds = c->p.vehicle == 1
                 ? solve8_lds_bytes(c->shape.lanes, c->p.T)
                 : solve_lds_bytes(c->shape.lanes, c->p.T, c->shape.ppl, c->shape.split, rs,
                                   c->p.n_con > 0);
    c->desc.rec_lds = records_on_chip(c, c->lds) ? 1 : 0;
    if (c->desc.rec_lds) c->lds += record_lds_bytes(c->shape.lanes, c->p.T, c->p.n_con);
    // static leading fields only: the device state is left as it is
    hipError_t e = hipMemcpy(c->d_desc, &c->desc, offsetof(InstanceDesc, cur),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    const std::vector<BlockDesc> tab = block_table(0, c->p.K, c->shape.lanes);
    return hipMemcpy(c->d_blocks, tab.data(), tab.size() * sizeof(BlockDesc),
                     hipMemcpyHostToDevice);
}

// stream the context's work is on (the batch's while it belongs to one)
hipStream_t work_stream(const bss_ctx* c) { return c->batch ? c->batch->stream : c->stream; }

// device state fields (cur, vshift, solve_index, done) of a context; while the context belongs to
// a batch they live in the batch's descriptor array
hipError_t read_state(bss_ctx* c, int32_t* st)
{
    const char* src = c->batch ? (const char*)(c->batch->d_desc + c->batch_index)
                               : (const char*)c->d_desc;
    const hipStream_t s = work_stream(c);
    hipError_t e = hipMemcpyAsync(c->host, src + kStateOffset, kStateBytes,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) std::memcpy(st, c->host, kStateBytes);
    return e;
}

hipError_t write_state(bss_ctx* c, const int32_t* st)
{
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
        e = hipMemcpy((char*)c->d_desc + kStateOffset, st, kStateBytes, hipMemcpyHostToDevice);
    return e;
}

}  // namespace

extern "C" {

void bss_params_default(bss_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->m = 1500.0;
    p->Iz = 2500.0;
    p->lf = 1.2;
    p->lr = 1.6;
    p->Cf = 5.0e4;
    p->Cr = 5.0e4;
    p->mu = 1.0;
    p->g = 9.81;
    p->v_min = 3.0;
    p->dt = 0.05;
    p->steer_max = 0.4;
    p->accel_max = 4.0;
    p->sigma_eps[0] = 0.1;
    p->sigma_eps[1] = 1.0;
    p->sigma_w[0] = 0.1;
    p->sigma_w[1] = 0.1;
    p->sigma_w[2] = 0.05;
    p->K = 256;
    p->M = 16;
    p->T = 30;
    p->delta = 0.05;
    p->gamma = 0.2;
    p->backoff = 0;
    p->belief = 0;
    p->crn = 0;
    p->sigma_w_speed = 0.0;
    p->n_obs = 0;
    for (int i = 0; i < 12; ++i) p->obs[i] = 0.0;
    p->local_repair = 0;
    p->n_con = 0;
    for (int i = 0; i < 6 * kMaxCon; ++i) p->con_a[i] = 0.0;
    for (int i = 0; i < kMaxCon; ++i) p->con_b[i] = 0.0;
    // the 8-state vehicle's values (used with vehicle = 1 only)
    p->vehicle = 0;
    p->Rw = 0.095;
    p->Iw = 0.3;
    p->T_max = 8.0;
    p->pac_B = 10.0;
    p->pac_C = 1.9;
    p->pac_D = 1.0;
    p->pac_E = 0.97;
    p->track_len = 120.0;
    p->kappa_amp = 0.8;
    p->n_sub = 4;
    p->lambda = 1.0;
    p->gamma_u = 1.0;
    p->v_goal = 6.0;
    p->q_vx = 1.0;
    p->q_vy = 0.0;
    p->q_r = 0.0;
    p->q_ey = 0.1;
    p->q_epsi = 1.0;
    p->C_cbf = 100.0;
    p->C_obs = 1000.0;
    p->phi_scale = 1.0;
    p->ell_a = 30.0;
    p->ell_b = 20.0;
    p->half_width = 2.0;
    p->shield_iters = 0;
    p->shield_gmin = 0.05;
    p->shield_fd = 1e-2;
    p->seed = 1;
    p->lanes = 0;
}

bss_status bss_validate(const bss_params* p)
{
    if (!p) return fail(BSS_E_INVAL, "params is NULL");
    if (p->K < 1 || p->K > (1 << 20)) return fail(BSS_E_INVAL, "K=%d outside [1, 2^20]", p->K);
    if (p->M < 1 || p->M > 512) return fail(BSS_E_INVAL, "M=%d outside [1, 512]", p->M);
    if (p->T < 1 || p->T > kMaxT) return fail(BSS_E_INVAL, "T=%d outside [1, %d]", p->T, kMaxT);
    if (!(p->delta > 0.0 && p->delta < 0.5))
        return fail(BSS_E_INVAL, "delta=%g outside (0, 0.5)", p->delta);
    if (!(p->gamma > 0.0 && p->gamma <= 1.0))
        return fail(BSS_E_INVAL, "gamma=%g outside (0, 1]", p->gamma);
    if (p->backoff != 0 && p->backoff != 1) return fail(BSS_E_INVAL, "backoff must be 0 or 1");
    if (p->belief < 0 || p->belief > 2) return fail(BSS_E_INVAL, "belief must be 0, 1 or 2");
    if (p->belief == 2 && p->M != 12)
        return fail(BSS_E_INVAL, "the sigma-point belief (belief = 2) uses M = 12 points");
    if (p->crn != 0 && p->crn != 1) return fail(BSS_E_INVAL, "crn must be 0 or 1");
    if (p->n_obs < 0 || p->n_obs > kMaxObstacles)
        return fail(BSS_E_INVAL, "n_obs must be 0..%d", kMaxObstacles);
    for (int i = 0; i < p->n_obs; ++i)
        if (!std::isfinite(p->obs[3 * i]) || !std::isfinite(p->obs[3 * i + 1]) ||
            !finite_pos(p->obs[3 * i + 2]))
            return fail(BSS_E_INVAL, "obstacle %d needs a finite centre and a radius > 0", i);
    if (!finite_nonneg(p->sigma_w_speed))
        return fail(BSS_E_INVAL, "sigma_w_speed must be finite and >= 0");
    if (p->local_repair < 0 || p->local_repair > 2)
        return fail(BSS_E_INVAL, "local_repair must be 0, 1 or 2");
    if (p->n_con < 0 || p->n_con > kMaxCon)
        return fail(BSS_E_INVAL, "n_con must be 0..%d", kMaxCon);
    for (int i = 0; i < p->n_con; ++i) {
        for (int j = 0; j < 6; ++j)
            if (!std::isfinite(p->con_a[6 * i + j]))
                return fail(BSS_E_INVAL, "half-space constraint %d: a must be finite", i);
        if (!std::isfinite(p->con_b[i]))
            return fail(BSS_E_INVAL, "half-space constraint %d: b must be finite", i);
    }
    if (!finite_pos(p->lambda)) return fail(BSS_E_INVAL, "lambda must be finite and > 0");
    if (!finite_pos(p->dt)) return fail(BSS_E_INVAL, "dt must be finite and > 0");
    if (!finite_pos(p->m) || !finite_pos(p->Iz) || !finite_pos(p->lf) || !finite_pos(p->lr))
        return fail(BSS_E_INVAL, "m, Iz, lf, lr must be finite and > 0");
    if (!finite_nonneg(p->Cf) || !finite_nonneg(p->Cr) || !finite_nonneg(p->mu) ||
        !finite_nonneg(p->g) || !finite_pos(p->v_min))
        return fail(BSS_E_INVAL, "Cf, Cr, mu, g must be >= 0 and v_min > 0");
    if (!finite_pos(p->steer_max) || !finite_pos(p->accel_max))
        return fail(BSS_E_INVAL, "control bounds must be finite and > 0");
    for (int i = 0; i < 2; ++i)
        if (!finite_nonneg(p->sigma_eps[i])) return fail(BSS_E_INVAL, "sigma_eps must be >= 0");
    for (int i = 0; i < 3; ++i)
        if (!finite_nonneg(p->sigma_w[i])) return fail(BSS_E_INVAL, "sigma_w must be >= 0");
    const double costs[] = {p->gamma_u, p->v_goal, p->q_vx, p->q_vy, p->q_r, p->q_ey,
                            p->q_epsi, p->C_cbf, p->C_obs, p->phi_scale};
    for (double c : costs)
        if (!std::isfinite(c)) return fail(BSS_E_INVAL, "cost weights must be finite");
    if (!finite_pos(p->ell_a) || !finite_pos(p->ell_b) || !finite_pos(p->half_width))
        return fail(BSS_E_INVAL, "track semi-axes and half-width must be > 0");
    {
        const double lo = std::fmin(p->ell_a, p->ell_b), hi = std::fmax(p->ell_a, p->ell_b);
        if (!(lo * lo / hi > p->half_width))
            return fail(BSS_E_INVAL,
                        "track: min(a,b)^2/max(a,b)=%g must exceed the half-width %g",
                        lo * lo / hi, p->half_width);
    }
    if (p->shield_iters < 0 || p->shield_iters > 16)
        return fail(BSS_E_INVAL, "shield_iters outside [0, 16]");
    if (p->local_repair != 0 && p->shield_iters < 1)
        return fail(BSS_E_INVAL, "the repair of the update (local_repair) needs shield_iters >= 1");
    if (p->shield_iters > 0 && (!finite_pos(p->shield_fd) || !finite_nonneg(p->shield_gmin)))
        return fail(BSS_E_INVAL, "shield_fd must be > 0 and shield_gmin >= 0");
    if (p->vehicle != 0 && p->vehicle != 1) return fail(BSS_E_INVAL, "vehicle must be 0 or 1");
    if (p->vehicle == 1) {
        if (!finite_pos(p->Rw) || !finite_pos(p->Iw) || !finite_nonneg(p->T_max))
            return fail(BSS_E_INVAL, "vehicle 1: Rw, Iw must be > 0 and T_max >= 0");
        if (!finite_pos(p->pac_B) || !finite_pos(p->pac_C) || !finite_pos(p->pac_D) ||
            !std::isfinite(p->pac_E))
            return fail(BSS_E_INVAL, "vehicle 1: magic-formula B, C, D must be > 0, E finite");
        if (!(p->track_len > 0.0) || !(std::fabs(p->kappa_amp) < 1.0))
            return fail(BSS_E_INVAL, "vehicle 1: track_len must be > 0 and |kappa_amp| < 1");
        const double kmax = 2.0 * M_PI / p->track_len * (1.0 + std::fabs(p->kappa_amp));
        if (!(2.0 * kmax * p->half_width < 1.0))
            return fail(BSS_E_INVAL, "vehicle 1: the road frame needs 2 w_T max|kappa| < 1 "
                                     "(got %g)", 2.0 * kmax * p->half_width);
        if (p->n_sub < 1 || p->n_sub > 64)
            return fail(BSS_E_INVAL, "vehicle 1: n_sub must be 1..64");
        if (p->shield_iters != 0 || p->n_obs != 0 || p->n_con != 0 || p->belief != 0 ||
            p->sigma_w_speed != 0.0 || p->local_repair != 0)
            return fail(BSS_E_INVAL, "vehicle 1 supports neither the repair, obstacles, "
                                     "half-space constraints, belief != 0, sigma_w_speed nor "
                                     "local_repair");
    }
    if (p->lanes != 0 && p->lanes != 8 && p->lanes != 16 && p->lanes != 32 && p->lanes != 64)
        return fail(BSS_E_INVAL, "lanes must be 0, 8, 16, 32 or 64");
    if (p->lanes != 0 && (p->M + p->lanes - 1) / p->lanes > 8)
        return fail(BSS_E_INVAL, "lanes=%d leaves more than 8 particles per lane for M=%d",
                    p->lanes, p->M);
    return BSS_OK;
}

bss_status bss_backoff(const bss_params* p, double* nu_out)
{
    bss_status st = bss_validate(p);
    if (st != BSS_OK) return st;
    if (!nu_out) return fail(BSS_E_INVAL, "nu_out is NULL");
    *nu_out = backoff_of(*p);
    return BSS_OK;
}

bss_status bss_create(const bss_params* p, const bss_allocator* alloc, void* stream,
                      bss_ctx** out)
{
    if (!out) return fail(BSS_E_INVAL, "out is NULL");
    *out = nullptr;
    bss_status st = bss_validate(p);
    if (st != BSS_OK) return st;
    if (alloc && (!alloc->alloc || !alloc->release))
        return fail(BSS_E_INVAL, "allocator must provide alloc and release");

    bss_ctx* c = new (std::nothrow) bss_ctx();
    if (!c) return fail(BSS_E_NOMEM, "host allocation failed");
    c->p = *p;
    c->has_alloc = alloc != nullptr;
    if (alloc) c->alloc = *alloc;
    c->stream = (hipStream_t)stream;
    c->shape = choose_shape(p->K, p->M, p->T, p->lanes, 0, -1, shape_for_shield(*p));
    c->timing = false;
    c->ev_used = 0;
    c->pending_shift = 0;
    c->outputs = BSS_OUT_CONTROLS | BSS_OUT_BELIEFS;
    c->batch = nullptr;
    c->batch_index = 0;
    c->host = nullptr;

    const size_t K = (size_t)p->K, T = (size_t)p->T;
    const size_t G = max_blocks(p->K);
    const size_t sz_v = align256(T * 2 * sizeof(double));
    const size_t sz_u = align256(K * T * 2 * sizeof(float));
    const size_t sz_mom = align256(K * (T + 1) * 9 * sizeof(double));
    const size_t sz_cvar = align256(K * (T + 1) * (size_t)p->n_con * sizeof(double));
    const size_t sz_S = align256(K * sizeof(double));
    const size_t sz_stats = align256(8 * sizeof(double));
    const size_t sz_part = align256(G * partial_stride(T) * sizeof(double));
    const size_t sz_x0 = 256;
    const size_t sz_sig = align256(36 * sizeof(double));
    const size_t sz_desc = align256(sizeof(InstanceDesc));
    const size_t sz_blk = align256(G * sizeof(BlockDesc));
    const size_t sz_col = align256(2 * T * sizeof(MergeDesc));
    // repair of the update: descriptor, grid, controls [T][2] f32, beliefs [T+1][9], constraint
    // variances [T+1][n_con], cost, partial [2T+5], stats [8]
    const size_t sz_rep = p->local_repair == 0
                              ? 0
                              : sz_desc + 256 + align256(T * 2 * sizeof(float)) +
                                    align256((T + 1) * 9 * sizeof(double)) +
                                    align256((T + 1) * (size_t)p->n_con * sizeof(double)) + 256 +
                                    align256(partial_stride(T) * sizeof(double)) + sz_stats;
    const size_t total = 2 * sz_v + sz_u + sz_mom + sz_cvar + sz_S + sz_stats + sz_part + sz_x0 +
                         sz_sig + sz_desc + sz_blk + sz_col + sz_rep;

    void* block = nullptr;
    if (c->has_alloc) {
        block = c->alloc.alloc(total, c->alloc.user);
        if (!block) {
            delete c;
            return fail(BSS_E_NOMEM, "allocator returned NULL for %zu bytes", total);
        }
    } else {
        hipError_t e = hipMalloc(&block, total);
        if (e != hipSuccess) {
            delete c;
            return fail(BSS_E_NOMEM, "hipMalloc(%zu): %s", total, hipGetErrorString(e));
        }
    }
    c->block = block;
    char* b = (char*)block;
    fill_desc(c);
    c->desc.v[0] = (double*)b;
    b += sz_v;
    c->desc.v[1] = (double*)b;
    b += sz_v;
    c->desc.u = (float*)b;
    b += sz_u;
    c->desc.mom = (double*)b;
    b += sz_mom;
    c->desc.cvar = p->n_con > 0 ? (double*)b : nullptr;
    b += sz_cvar;
    c->desc.S = (double*)b;
    b += sz_S;
    c->desc.stats = (double*)b;
    b += sz_stats;
    c->desc.partial = (double*)b;
    b += sz_part;
    c->x0 = (double*)b;
    b += sz_x0;
    c->Sigma0 = (double*)b;
    b += sz_sig;
    c->d_desc = (InstanceDesc*)b;
    b += sz_desc;
    c->d_blocks = (BlockDesc*)b;
    b += sz_blk;
    c->d_cols = (MergeDesc*)b;
    b += sz_col;
    c->d_rdesc = nullptr;
    c->d_rblock = nullptr;
    c->rlds = 0;
    if (p->local_repair != 0) {
        // one sample, no exploration noise, its own Philox key (seed ^ 0x5DEECE66DA3B9F1B, sample
        // word 0) and buffers; both mean-sequence pointers are the context's
        InstanceDesc& r = c->rdesc;
        r = c->desc;
        r.K = 1;
        r.nblocks = 1;
        r.sig_eps0 = 0.0f;
        r.sig_eps1 = 0.0f;
        r.shift_after = 0;
        const uint64_t rkey = p->seed ^ 0x5DEECE66DA3B9F1Bull;
        r.key0 = (uint32_t)rkey;
        r.key1 = (uint32_t)(rkey >> 32);
        c->d_rdesc = (InstanceDesc*)b;
        b += sz_desc;
        c->d_rblock = (BlockDesc*)b;
        b += 256;
        r.u = (float*)b;
        b += align256(T * 2 * sizeof(float));
        r.mom = (double*)b;
        b += align256((T + 1) * 9 * sizeof(double));
        r.cvar = p->n_con > 0 ? (double*)b : nullptr;
        b += align256((T + 1) * (size_t)p->n_con * sizeof(double));
        r.sc.shield_iters = p->shield_iters;   // the repair pass always repairs
        r.S = (double*)b;
        b += 256;
        r.partial = (double*)b;
        b += align256(partial_stride(T) * sizeof(double));
        r.stats = (double*)b;
        // a single sample is latency-bound: as many lanes as the particles can use (up to the
        // wave), so that each lane steps few particles, whatever the shape of the sampled solve
        c->rshape = choose_shape(1, p->M, p->T, 0, 1, 0, true);
        r.lanes = c->rshape.lanes;
        r.ppl = c->rshape.ppl;
        r.rec_lds = 0;
        c->rlds = solve_lds_bytes(r.lanes, p->T, c->rshape.ppl, false, false, p->n_con > 0);
    }

    hipError_t e = hipHostMalloc((void**)&c->host, 64 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        c->host = nullptr;
        bss_destroy(c);
        return fail(BSS_E_NOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    // zero every buffer (warm start, stats), then the descriptors and grids
    e = hipMemsetAsync(block, 0, total, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
        e = hipMemcpy(c->d_desc, &c->desc, sizeof(InstanceDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess && c->d_rdesc) {
        const BlockDesc rb{0, 0};
        e = hipMemcpy(c->d_rdesc, &c->rdesc, sizeof(InstanceDesc), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(c->d_rblock, &rb, sizeof(BlockDesc), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = upload_shape(c);
    if (e == hipSuccess) {
        std::vector<MergeDesc> cols;
        for (int col = 0; col < 2 * p->T; ++col) cols.push_back(MergeDesc{0, col});
        e = hipMemcpy(c->d_cols, cols.data(), cols.size() * sizeof(MergeDesc),
                      hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        bss_destroy(c);
        return device_fail(e, "initialising context buffers");
    }
    *out = c;
    return BSS_OK;
}

bss_status bss_set_stream(bss_ctx* c, void* stream)
{
    if (!c) return fail(BSS_E_INVAL, "ctx is NULL");
    c->stream = (hipStream_t)stream;
    return BSS_OK;
}

static bss_status check_free(const bss_ctx* c)
{
    if (!c) return fail(BSS_E_INVAL, "ctx is NULL");
    if (c->batch) return fail(BSS_E_STATE, "context belongs to a batch (bss_batch_destroy first)");
    return BSS_OK;
}

static bss_status enqueue_solve(bss_ctx* c, const double* x0_dev, const double* Sigma0_dev)
{
    hipError_t e;
    if (c->timing) {
        if (c->ev_used + 2 > c->ev.size()) {
            for (int i = 0; i < 64; ++i) {
                // timing only (read after a stream synchronisation): no system-scope fence, so
                // a record does not write back and invalidate the caches between the launches
                hipEvent_t ev;
                e = hipEventCreateWithFlags(&ev, hipEventDisableSystemFence);
                if (e != hipSuccess) return device_fail(e, "hipEventCreateWithFlags");
                c->ev.push_back(ev);
            }
        }
        e = hipEventRecord(c->ev[c->ev_used], c->stream);
        if (e != hipSuccess) return device_fail(e, "hipEventRecord");
    }
    if (c->p.vehicle == 1) {
        if (Sigma0_dev)
            return fail(BSS_E_INVAL, "vehicle 1 takes a known estimate (Sigma0 must be NULL)");
        e = launch_solve8(c->d_desc, c->d_blocks, c->desc.nblocks, c->shape.ppl, c->lds, x0_dev,
                          c->pending_shift, c->stream);
    } else {
        e = launch_solve(c->d_desc, c->d_blocks, c->desc.nblocks, c->shape.ppl,
                         launch_shield(c->p), c->shape.split, launch_resample(c->p),
                         c->p.n_con > 0, c->lds, x0_dev, Sigma0_dev, c->pending_shift,
                         c->stream);
    }
    if (e != hipSuccess) return device_fail(e, "solve launch");
    if (c->timing) {
        e = hipEventRecord(c->ev[c->ev_used + 1], c->stream);
        if (e != hipSuccess) return device_fail(e, "hipEventRecord");
        c->ev_used += 2;
    }
    e = launch_merge(c->d_desc, c->d_cols, 2 * c->p.T, c->pending_shift, c->stream);
    if (e != hipSuccess) return device_fail(e, "merge launch");
    c->pending_shift = 0;
    if (c->d_rdesc) {
        e = launch_local_repair(c->d_desc, c->d_rdesc, c->d_rblock, c->p.T, c->rshape.ppl,
                                launch_resample(c->p), c->p.n_con > 0, c->rlds, x0_dev,
                                Sigma0_dev, c->stream);
        if (e != hipSuccess) return device_fail(e, "repair of the update");
    }
    return BSS_OK;
}

bss_status bss_solve_async(bss_ctx* c, const double* x0_dev, const double* Sigma0_dev)
{
    bss_status st = check_free(c);
    if (st != BSS_OK) return st;
    if (!x0_dev) return fail(BSS_E_INVAL, "x0 is NULL");
    return enqueue_solve(c, x0_dev, Sigma0_dev);
}

static void fill_info(const bss_ctx* c, const double* stats, bss_info* info)
{
    if (!info) return;
    info->S_min = stats[0];
    info->Z = stats[1];
    info->ess = stats[2];
    info->n_finite = (int32_t)stats[3];
    info->dcbf_violations = (int32_t)stats[7];
    // the rollout kernel's time of the last solve (the stream is synchronised by the callers)
    info->kernel_ms = -1.0f;
    if (c->timing && !c->batch && c->ev_used >= 2) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->ev[c->ev_used - 2], c->ev[c->ev_used - 1]) == hipSuccess)
            info->kernel_ms = ms;
    }
    info->records_on_chip = c->batch ? 0 : c->desc.rec_lds;
    if (c->batch) {
        info->lanes = c->batch->lanes[c->batch_index];
        info->ppl = c->batch->ppls[c->batch_index];
        info->split = c->batch->split ? 1 : 0;
    } else {
        info->lanes = c->shape.lanes;
        info->ppl = c->shape.ppl;
        info->split = c->shape.split ? 1 : 0;
    }
}

bss_status bss_solve(bss_ctx* c, const double x0[6], const double* Sigma0, double u0_out[2],
                     bss_info* info)
{
    bss_status st = check_free(c);
    if (st != BSS_OK) return st;
    if (!x0 || !u0_out) return fail(BSS_E_INVAL, "x0 and u0_out must not be NULL");
    const int nx = c->p.vehicle == 1 ? 8 : 6;
    for (int i = 0; i < nx; ++i)
        if (!std::isfinite(x0[i])) return fail(BSS_E_INVAL, "x0[%d] is not finite", i);
    if (Sigma0 && c->p.vehicle == 1)
        return fail(BSS_E_INVAL, "vehicle 1 takes a known estimate (Sigma0 must be NULL)");
    if (Sigma0) {
        for (int i = 0; i < 36; ++i)
            if (!std::isfinite(Sigma0[i])) return fail(BSS_E_INVAL, "Sigma0[%d] not finite", i);
        for (int i = 0; i < 6; ++i)
            if (Sigma0[i * 6 + i] < 0.0) return fail(BSS_E_INVAL, "Sigma0 has a negative variance");
    }
    // stage through pinned memory so the copies are truly asynchronous
    std::memcpy(c->host + 16, x0, nx * sizeof(double));
    if (Sigma0) std::memcpy(c->host + 24, Sigma0, 36 * sizeof(double));
    hipError_t e = hipMemcpyAsync(c->x0, c->host + 16, nx * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && Sigma0)
        e = hipMemcpyAsync(c->Sigma0, c->host + 24, 36 * sizeof(double), hipMemcpyHostToDevice,
                           c->stream);
    if (e != hipSuccess) return device_fail(e, "staging x0");
    st = enqueue_solve(c, c->x0, Sigma0 ? c->Sigma0 : nullptr);
    if (st != BSS_OK) return st;
    e = hipMemcpyAsync(c->host, c->desc.stats, 8 * sizeof(double), hipMemcpyDeviceToHost,
                       c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_fail(e, "solve");
    fill_info(c, c->host, info);
    u0_out[0] = c->host[5];
    u0_out[1] = c->host[6];
    if (c->host[4] != 0.0) return fail(BSS_E_NUMERIC, "no sample had a finite cost");
    return BSS_OK;
}

bss_status bss_step_shift(bss_ctx* c)
{
    bss_status st = check_free(c);
    if (st != BSS_OK) return st;
    if (c->pending_shift < c->p.T - 1) c->pending_shift += 1;
    return BSS_OK;
}

bss_status bss_set_outputs(bss_ctx* c, int32_t flags)
{
    bss_status st = check_free(c);
    if (st != BSS_OK) return st;
    if (flags & ~(BSS_OUT_CONTROLS | BSS_OUT_BELIEFS)) return fail(BSS_E_INVAL, "unknown flags");
    c->outputs = flags;
    float* u = (flags & BSS_OUT_CONTROLS) ? (float*)((char*)c->desc.v[1] +
                                                     align256((size_t)c->p.T * 2 * sizeof(double)))
                                          : nullptr;
    c->desc.u = u;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
        e = hipMemcpy((char*)c->d_desc + offsetof(InstanceDesc, u), &u, sizeof(u),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = upload_shape(c);   // where the records live, and the LDS
    if (e != hipSuccess) return device_fail(e, "setting outputs");
    return BSS_OK;
}

bss_status bss_get_buffers(const bss_ctx* cc, bss_buffers* out)
{
    bss_ctx* c = const_cast<bss_ctx*>(cc);
    if (!c || !out) return fail(BSS_E_INVAL, "NULL argument");
    int32_t stv[4];
    hipError_t e = read_state(c, stv);
    if (e != hipSuccess) return device_fail(e, "reading state");
    const int cur = stv[0];
    out->v = c->desc.v[cur];
    out->u = (float*)((char*)c->desc.v[1] + align256((size_t)c->p.T * 2 * sizeof(double)));
    out->mom = c->desc.mom;
    out->con_var = c->desc.cvar;
    out->S = c->desc.S;
    out->stats = c->desc.stats;
    out->x0 = c->x0;
    out->Sigma0 = c->Sigma0;
    out->v_shift = stv[1] + c->pending_shift;
    return BSS_OK;
}

bss_status bss_get_controls(bss_ctx* c, double* v_host)
{
    if (!c || !v_host) return fail(BSS_E_INVAL, "NULL argument");
    int32_t stv[4];
    hipError_t e = read_state(c, stv);
    if (e != hipSuccess) return device_fail(e, "reading state");
    const int T = c->p.T;
    const int shift = stv[1] + c->pending_shift;
    std::vector<double> tmp((size_t)T * 2);
    e = hipMemcpy(tmp.data(), c->desc.v[stv[0]], (size_t)T * 2 * sizeof(double),
                  hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_fail(e, "reading controls");
    for (int t = 0; t < T; ++t) {
        const int r = t + shift < T ? t + shift : T - 1;
        v_host[2 * t] = tmp[2 * r];
        v_host[2 * t + 1] = tmp[2 * r + 1];
    }
    return BSS_OK;
}

bss_status bss_set_controls(bss_ctx* c, const double* v_host)
{
    bss_status st = check_free(c);
    if (st != BSS_OK) return st;
    if (!v_host) return fail(BSS_E_INVAL, "NULL argument");
    for (int i = 0; i < 2 * c->p.T; ++i)
        if (!std::isfinite(v_host[i])) return fail(BSS_E_INVAL, "controls must be finite");
    int32_t stv[4];
    hipError_t e = read_state(c, stv);
    if (e == hipSuccess)
        e = hipMemcpy(c->desc.v[stv[0]], v_host, (size_t)c->p.T * 2 * sizeof(double),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        stv[1] = 0;
        e = write_state(c, stv);
    }
    if (e != hipSuccess) return device_fail(e, "writing controls");
    c->pending_shift = 0;
    return BSS_OK;
}

bss_status bss_set_solve_index(bss_ctx* c, uint32_t s)
{
    bss_status st = check_free(c);
    if (st != BSS_OK) return st;
    int32_t stv[4];
    hipError_t e = read_state(c, stv);
    if (e == hipSuccess) {
        stv[2] = (int32_t)s;
        e = write_state(c, stv);
    }
    if (e != hipSuccess) return device_fail(e, "writing solve index");
    return BSS_OK;
}

bss_status bss_get_solve_index(const bss_ctx* cc, uint32_t* s)
{
    bss_ctx* c = const_cast<bss_ctx*>(cc);
    if (!c || !s) return fail(BSS_E_INVAL, "NULL argument");
    int32_t stv[4];
    hipError_t e = read_state(c, stv);
    if (e != hipSuccess) return device_fail(e, "reading solve index");
    *s = (uint32_t)stv[2];
    return BSS_OK;
}

bss_status bss_get_info(bss_ctx* c, bss_info* info)
{
    if (!c || !info) return fail(BSS_E_INVAL, "NULL argument");
    const hipStream_t s = work_stream(c);
    hipError_t e = hipMemcpyAsync(c->host, c->desc.stats, 8 * sizeof(double),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(e, "reading stats");
    fill_info(c, c->host, info);
    return BSS_OK;
}

bss_status bss_timing_enable(bss_ctx* c, int32_t enable)
{
    if (!c) return fail(BSS_E_INVAL, "ctx is NULL");
    c->timing = enable != 0;
    return BSS_OK;
}

bss_status bss_timing_read(bss_ctx* c, double* rollout_ms_total, int32_t* count)
{
    if (!c || !rollout_ms_total || !count) return fail(BSS_E_INVAL, "NULL argument");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_fail(e, "synchronising");
    double total = 0.0;
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]);
        if (e != hipSuccess) return device_fail(e, "hipEventElapsedTime");
        total += ms;
    }
    *rollout_ms_total = total;
    *count = (int32_t)(c->ev_used / 2);
    c->ev_used = 0;
    return BSS_OK;
}

bss_status bss_set_shape(bss_ctx* c, int32_t lanes, int32_t ppl, int32_t split)
{
    bss_status st = check_free(c);
    if (st != BSS_OK) return st;
    bss_params q = c->p;
    q.lanes = lanes;
    st = bss_validate(&q);
    if (st != BSS_OK) return st;
    if (ppl != 0 && ppl != 1 && ppl != 2 && ppl != 4 && ppl != 8)
        return fail(BSS_E_INVAL, "particles per lane must be 0, 1, 2, 4 or 8");
    if (ppl != 0 && (q.M + ppl - 1) / ppl > 64)
        return fail(BSS_E_INVAL, "M=%d needs more than 64 lanes with %d particles per lane", q.M,
                    ppl);
    if (split < -1 || split > 1) return fail(BSS_E_INVAL, "split must be -1, 0 or 1");
    const LaunchShape sh = choose_shape(q.K, q.M, q.T, lanes, ppl, split, shape_for_shield(q));
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_fail(e, "synchronising");
    c->shape = sh;
    e = upload_shape(c);
    if (e != hipSuccess) return device_fail(e, "uploading launch shape");
    return BSS_OK;
}

bss_status bss_set_lanes(bss_ctx* c, int32_t lanes) { return bss_set_shape(c, lanes, 0, -1); }

void bss_destroy(bss_ctx* c)
{
    if (!c) return;
    if (c->batch) return;   // owned by a batch: bss_batch_destroy releases it first
    (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t ev : c->ev) (void)hipEventDestroy(ev);
    if (c->block) {
        if (c->has_alloc) c->alloc.release(c->block, c->alloc.user);
        else (void)hipFree(c->block);
    }
    if (c->host) (void)hipHostFree(c->host);
    delete c;
}

// ---- batches ---------------------------------------------------------------------------------
static hipError_t batch_layout(bss_batch* b, int ppl, int split)
{
    // launch shape of every instance for a common particles-per-lane count (ppl > 0) or for each
    // member's own (ppl == 0, b->member_ppl), the solve grid with blocks ordered by their work
    // (longest first: every thread of a block steps P particles for T steps), and the merge grid
    std::vector<BlockDesc> blocks;
    std::vector<MergeDesc> cols;
    std::vector<int> lanes(b->n), ppls(b->n);
    size_t lds = 0;
    for (int i = 0; i < b->n; ++i) {
        const bss_params& p = b->ctxs[i]->p;
        ppls[i] = ppl != 0 ? ppl : b->member_ppl[i];
        const LaunchShape sh = choose_shape(p.K, p.M, p.T, 0, ppls[i], 0);
        lanes[i] = sh.lanes;
        std::vector<BlockDesc> t = block_table(i, p.K, sh.lanes);
        blocks.insert(blocks.end(), t.begin(), t.end());
        for (int col = 0; col < 2 * p.T; ++col) cols.push_back(MergeDesc{i, col});
    }
    std::stable_sort(blocks.begin(), blocks.end(), [&](const BlockDesc& x, const BlockDesc& y) {
        return (int64_t)b->ctxs[x.inst]->p.T * ppls[x.inst] >
               (int64_t)b->ctxs[y.inst]->p.T * ppls[y.inst];
    });
    // split blocks (noise generated by a second set of waves) when asked, or automatically when
    // the whole grid has fewer than two waves per SIMD; every member's ring must fit
    bool sp = split > 0 || (split < 0 && (int64_t)blocks.size() * 4 < 2 * 1024);
    sp = sp && !b->shield && !b->resample;
    for (int i = 0; i < b->n && sp; ++i)
        sp = solve_base_lds_bytes(lanes[i], b->ctxs[i]->p.T, ppls[i], true) <= kMaxLds &&
             split_fits(lanes[i], b->ctxs[i]->p.T, ppls[i], false, b->con, kStaticLdsSlots);
    for (int i = 0; i < b->n; ++i)
        lds = std::max(lds, solve_lds_bytes(lanes[i], b->ctxs[i]->p.T, ppls[i], sp,
                                            b->resample, b->con));
    hipError_t e = hipSuccess;
    for (int i = 0; i < b->n && e == hipSuccess; ++i) {
        InstanceDesc head = b->ctxs[i]->desc;
        head.lanes = lanes[i];
        head.ppl = ppls[i];
        head.rec_lds = 0;   // a batch keeps every member's records in HBM
        head.nblocks = solve_blocks(b->ctxs[i]->p.K, lanes[i]);
        head.x0_index = i;
        e = hipMemcpy(b->d_desc + i, &head, offsetof(InstanceDesc, cur), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess)
        e = hipMemcpy(b->d_blocks, blocks.data(), blocks.size() * sizeof(BlockDesc),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_cols, cols.data(), cols.size() * sizeof(MergeDesc),
                      hipMemcpyHostToDevice);
    b->nblocks = (int)blocks.size();
    b->ncols = (int)cols.size();
    b->lds = lds;
    b->ppl = ppl;
    b->split = sp;
    b->lanes = lanes;
    b->ppls = ppls;
    return e;
}

static hipError_t batch_enqueue(bss_batch* b)
{
    hipError_t e = launch_solve(b->d_desc, b->d_blocks, b->nblocks, b->ppl, b->shield,
                                b->split, b->resample, b->con, b->lds,
                                b->d_x0, nullptr, 0, b->stream,
                                b->persistent ? b->d_queue : nullptr);
    if (e == hipSuccess) e = launch_merge(b->d_desc, b->d_cols, b->ncols, 0, b->stream);
    return e;
}

static void batch_free(bss_batch* b)
{
    if (b->captured) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
    }
    if (b->block) (void)hipFree(b->block);
    for (bss_ctx* c : b->ctxs)
        if (c && c->batch == b) c->batch = nullptr;
    delete b;
}

bss_status bss_batch_create(bss_ctx* const* ctxs, int32_t n, int32_t ppl, int32_t shift_after,
                            bss_batch** out)
{
    if (!out) return fail(BSS_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!ctxs || n < 1) return fail(BSS_E_INVAL, "need at least one context");
    if (ppl != 0 && ppl != 1 && ppl != 2 && ppl != 4 && ppl != 8)
        return fail(BSS_E_INVAL, "particles per lane must be 0 (tune), 1, 2, 4 or 8");
    if (shift_after != 0 && shift_after != 1) return fail(BSS_E_INVAL, "shift_after must be 0/1");
    int M_max = 0;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return fail(BSS_E_INVAL, "context %d is NULL", i);
        if (ctxs[i]->batch) return fail(BSS_E_STATE, "context %d already belongs to a batch", i);
        if (ctxs[i]->p.vehicle != 0)
            return fail(BSS_E_INVAL, "context %d uses the 8-state vehicle, which batches do not "
                                     "run", i);
        if (ctxs[i]->p.local_repair != 0)
            return fail(BSS_E_INVAL, "context %d repairs its update (local_repair), which runs per "
                        "context, not in batches", i);
        for (int q = 0; q < i; ++q)
            if (ctxs[q] == ctxs[i]) return fail(BSS_E_INVAL, "context %d appears twice", i);
        M_max = std::max(M_max, ctxs[i]->p.M);
    }
    if (ppl != 0 && (M_max + ppl - 1) / ppl > 64)
        return fail(BSS_E_INVAL, "M=%d needs more than 64 lanes with %d particles per lane",
                    M_max, ppl);
    bss_batch* b = new (std::nothrow) bss_batch();
    if (!b) return fail(BSS_E_NOMEM, "host allocation failed");
    b->ctxs.assign(ctxs, ctxs + n);
    b->n = n;
    b->stream = ctxs[0]->stream;
    b->shift_after = shift_after;
    b->captured = false;
    b->block = nullptr;
    b->shield = false;
    b->resample = false;
    b->con = false;
    size_t nb = 0, nc = 0;
    for (int i = 0; i < n; ++i) {
        nb += max_blocks(ctxs[i]->p.K);
        nc += 2 * (size_t)ctxs[i]->p.T;
        b->shield = b->shield || launch_shield(ctxs[i]->p);
        b->resample = b->resample || launch_resample(ctxs[i]->p);
        b->con = b->con || ctxs[i]->p.n_con > 0;
    }
    const size_t sz_desc = align256((size_t)n * sizeof(InstanceDesc));
    const size_t total = 2 * sz_desc + align256(nb * sizeof(BlockDesc)) +
                         align256(nc * sizeof(MergeDesc)) +
                         align256((size_t)n * 6 * sizeof(double)) + 256;
    hipError_t e = hipMalloc(&b->block, total);
    if (e != hipSuccess) {
        b->block = nullptr;
        batch_free(b);
        return fail(BSS_E_NOMEM, "hipMalloc(%zu): %s", total, hipGetErrorString(e));
    }
    char* p = (char*)b->block;
    b->d_desc = (InstanceDesc*)p;
    p += sz_desc;
    b->d_backup = (InstanceDesc*)p;
    p += sz_desc;
    b->d_blocks = (BlockDesc*)p;
    p += align256(nb * sizeof(BlockDesc));
    b->d_cols = (MergeDesc*)p;
    p += align256(nc * sizeof(MergeDesc));
    b->d_x0 = (double*)p;
    p += align256((size_t)n * 6 * sizeof(double));
    b->d_queue = (uint32_t*)p;
    b->persistent = false;

    // the batch takes over each context's descriptor (device state included); pending host
    // shifts are folded into the device state
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        bss_ctx* c = ctxs[i];
        e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess)
            e = hipMemcpy(b->d_desc + i, c->d_desc, sizeof(InstanceDesc), hipMemcpyDeviceToDevice);
        if (e == hipSuccess) {
            int32_t sa[2] = {shift_after, 0};
            e = hipMemcpy((char*)(b->d_desc + i) + offsetof(InstanceDesc, shift_after), sa,
                          sizeof(sa), hipMemcpyHostToDevice);
        }
        if (e == hipSuccess && c->pending_shift) {
            int32_t stv[4];
            e = hipMemcpy(stv, (char*)(b->d_desc + i) + kStateOffset, kStateBytes,
                          hipMemcpyDeviceToHost);
            stv[1] = std::min(stv[1] + c->pending_shift, c->p.T - 1);
            if (e == hipSuccess)
                e = hipMemcpy((char*)(b->d_desc + i) + kStateOffset, stv, kStateBytes,
                              hipMemcpyHostToDevice);
            c->pending_shift = 0;
        }
    }
    if (e == hipSuccess) e = hipMemset(b->d_x0, 0, (size_t)n * 6 * sizeof(double));
    const int ppl0 = ppl != 0 ? ppl : (M_max > 256 ? 8 : 4);
    b->member_ppl.assign(n, ppl0);
    if (e == hipSuccess) e = batch_layout(b, ppl0, -1);
    if (e != hipSuccess) {
        batch_free(b);
        return device_fail(e, "creating batch");
    }
    for (int i = 0; i < n; ++i) {
        ctxs[i]->batch = b;
        ctxs[i]->batch_index = i;
    }
    *out = b;
    return BSS_OK;
}

bss_status bss_batch_states(bss_batch* b, double** x0_dev)
{
    if (!b || !x0_dev) return fail(BSS_E_INVAL, "NULL argument");
    *x0_dev = b->d_x0;
    return BSS_OK;
}

bss_status bss_batch_set_states(bss_batch* b, const double* x0_host)
{
    if (!b || !x0_host) return fail(BSS_E_INVAL, "NULL argument");
    for (int i = 0; i < 6 * b->n; ++i)
        if (!std::isfinite(x0_host[i])) return fail(BSS_E_INVAL, "state %d is not finite", i / 6);
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_x0, x0_host, (size_t)b->n * 6 * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return device_fail(e, "writing states");
    return BSS_OK;
}

bss_status bss_batch_copy_states(bss_batch* b, const double* x0_dev)
{
    if (!b || !x0_dev) return fail(BSS_E_INVAL, "NULL argument");
    hipError_t e = hipMemcpyAsync(b->d_x0, x0_dev, (size_t)b->n * 6 * sizeof(double),
                                  hipMemcpyDeviceToDevice, b->stream);
    if (e != hipSuccess) return device_fail(e, "copying states");
    return BSS_OK;
}

bss_status bss_batch_solve(bss_batch* b)
{
    if (!b) return fail(BSS_E_INVAL, "batch is NULL");
    hipError_t e = b->captured ? hipGraphLaunch(b->exec, b->stream) : batch_enqueue(b);
    if (e != hipSuccess) return device_fail(e, "batch solve");
    return BSS_OK;
}

bss_status bss_batch_capture(bss_batch* b)
{
    if (!b) return fail(BSS_E_INVAL, "batch is NULL");
    if (b->captured) return BSS_OK;
    if (b->stream == nullptr)
        return fail(BSS_E_STATE, "graph capture needs the batch on a created (non-null) stream");
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return device_fail(e, "hipStreamBeginCapture");
    hipError_t le = batch_enqueue(b);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->stream, &g);
    if (le != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return device_fail(le != hipSuccess ? le : e, "capturing the batch launch");
    }
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return device_fail(e, "hipGraphInstantiate");
    }
    b->graph = g;
    b->captured = true;
    return BSS_OK;
}

// Autotuning results per batch signature (the members' K, M, T and variant flags, in order) and
// device, for the life of the process.
struct TuneChoice {
    int ppl, split;
    bool persistent;
    std::vector<int> member_ppl;   // each member's P when ppl == 0
    float ms;
};

static std::mutex g_tune_mutex;
static std::map<std::string, TuneChoice> g_tune_cache;

static std::string tune_key(const bss_batch* b)
{
    int dev = -1;
    (void)hipGetDevice(&dev);
    std::string key = "dev" + std::to_string(dev);
    for (const bss_ctx* c : b->ctxs) {
        const bss_params& p = c->p;
        key += "|" + std::to_string(p.K) + "," + std::to_string(p.M) + "," + std::to_string(p.T) +
               "," + std::to_string(launch_shield(p)) + std::to_string(launch_resample(p)) +
               std::to_string(p.n_con > 0);
    }
    return key;
}

static bool plain_batch(const bss_batch* b) { return !b->shield && !b->resample && !b->con; }

// Lays the batch out (ppl 0: b->member_ppl) and times three solves after two warm-up solves;
// *applied is false when the layout could not take the requested noise split.
static hipError_t time_layout(bss_batch* b, int ppl, int split, bool persistent, hipEvent_t ev0,
                              hipEvent_t ev1, float* ms, bool* applied)
{
    b->persistent = persistent;
    hipError_t e = batch_layout(b, ppl, split);
    *applied = e == hipSuccess && (split == 1) == b->split;
    if (!*applied) return e;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) e = batch_enqueue(b);
    if (e == hipSuccess) e = hipEventRecord(ev0, b->stream);
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) e = batch_enqueue(b);
    if (e == hipSuccess) e = hipEventRecord(ev1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, ev0, ev1);
    return e;
}

static hipError_t apply_choice(bss_batch* b, const TuneChoice& t)
{
    b->persistent = t.persistent;
    if (t.ppl == 0) b->member_ppl = t.member_ppl;
    return batch_layout(b, t.ppl, t.split);
}

bss_status bss_batch_tune(bss_batch* b, int32_t* ppl_out)
{
    if (!b) return fail(BSS_E_INVAL, "batch is NULL");
    if (b->captured) return fail(BSS_E_STATE, "tune before capturing the batch");
    const std::string key = tune_key(b);
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            hipError_t e = apply_choice(b, it->second);
            if (e != hipSuccess) return device_fail(e, "applying the cached batch layout");
            if (ppl_out) *ppl_out = it->second.ppl;
            return BSS_OK;
        }
    }
    int M_max = 0;
    for (bss_ctx* c : b->ctxs) M_max = std::max(M_max, c->p.M);
    // the trial solves advance each member's state, overwrite both of its mean-sequence buffers
    // and its stats: save the descriptors, the buffers and the stats, restore them afterwards
    size_t vbytes = 0;
    for (bss_ctx* c : b->ctxs) vbytes += (2 * (size_t)c->p.T * 2 + 8) * sizeof(double);
    double* vsave = nullptr;
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = hipMalloc(&vsave, vbytes);
    if (e != hipSuccess) return device_fail(e, "allocating the tuning backup");
    auto copy_state = [&](bool save) {
        hipError_t r = hipSuccess;
        char* q = (char*)vsave;
        for (bss_ctx* c : b->ctxs) {
            const size_t nb = (size_t)c->p.T * 2 * sizeof(double);
            double* bufs[3] = {c->desc.v[0], c->desc.v[1], c->desc.stats};
            const size_t sizes[3] = {nb, nb, 8 * sizeof(double)};
            for (int h = 0; h < 3 && r == hipSuccess; ++h) {
                r = save ? hipMemcpy(q, bufs[h], sizes[h], hipMemcpyDeviceToDevice)
                         : hipMemcpy(bufs[h], q, sizes[h], hipMemcpyDeviceToDevice);
                q += sizes[h];
            }
        }
        return r;
    };
    e = copy_state(true);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_backup, b->d_desc, (size_t)b->n * sizeof(InstanceDesc),
                      hipMemcpyDeviceToDevice);
    if (e != hipSuccess) {
        (void)hipFree(vsave);
        return device_fail(e, "saving batch state");
    }
    hipEvent_t ev0, ev1;
    if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess) {
        (void)hipFree(vsave);
        return fail(BSS_E_DEVICE, "hipEventCreate");
    }
    const bool plain = plain_batch(b);
    const int cands[] = {1, 2, 4, 8};
    // 1. one P for every member: P x noise split x one-shot or persistent grid (the persistent
    //    grid and the per-member P exist for plain batches only)
    TuneChoice best{b->ppl, b->split ? 1 : 0, false, b->member_ppl, 1e30f};
    for (int cand : cands) {
        if ((M_max + cand - 1) / cand > 64) continue;
        for (int sp = 0; sp <= (plain ? 1 : 0) && e == hipSuccess; ++sp) {
            bool applied = true;
            for (int pers = 0; pers <= (plain ? 1 : 0) && e == hipSuccess && applied; ++pers) {
                float ms = 0.0f;
                e = time_layout(b, cand, sp, pers == 1, ev0, ev1, &ms, &applied);
                if (e == hipSuccess && applied && ms < best.ms)
                    best = TuneChoice{cand, sp, pers == 1, {}, ms};
            }
            if (!applied) break;   // the split ring does not fit this batch
        }
        if (e != hipSuccess) break;
    }
    // 2. each member's own P in one launch: members grouped by M (which sets how many of a
    //    layout's particle slots are used); starting from the best common P, the groups in order
    //    of their work try every other P, and a change is kept when the whole batch gets faster
    //    by more than 1 %
    if (plain && e == hipSuccess && best.ppl != 0) {
        std::vector<int> mp(b->n, best.ppl);
        b->member_ppl = mp;
        float cur = 0.0f;
        bool applied = false;
        e = time_layout(b, 0, best.split, best.persistent, ev0, ev1, &cur, &applied);
        if (e == hipSuccess && applied) {
            std::map<int, double> work;
            for (bss_ctx* c : b->ctxs) work[c->p.M] += (double)c->p.K * c->p.M * c->p.T;
            std::vector<std::pair<double, int>> order;
            for (const auto& kv : work) order.push_back({kv.second, kv.first});
            std::sort(order.rbegin(), order.rend());
            for (const auto& grp : order) {
                const int M = grp.second;
                int now = best.ppl;
                for (int i = 0; i < b->n; ++i)
                    if (b->ctxs[i]->p.M == M) now = mp[i];
                for (int cand : cands) {
                    if (cand == now || (M + cand - 1) / cand > 64) continue;
                    std::vector<int> trial = mp;
                    for (int i = 0; i < b->n; ++i)
                        if (b->ctxs[i]->p.M == M) trial[i] = cand;
                    b->member_ppl = trial;
                    float ms = 0.0f;
                    e = time_layout(b, 0, best.split, best.persistent, ev0, ev1, &ms, &applied);
                    if (e != hipSuccess) break;
                    if (applied && ms < 0.99f * cur) {
                        mp = trial;
                        cur = ms;
                        now = cand;
                    }
                }
                if (e != hipSuccess) break;
            }
            if (e == hipSuccess && cur < best.ms)
                best = TuneChoice{0, best.split, best.persistent, mp, cur};
        }
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    // restore the state the trial solves advanced, then the chosen layout
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_desc, b->d_backup, (size_t)b->n * sizeof(InstanceDesc),
                      hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = copy_state(false);
    (void)hipFree(vsave);
    if (e == hipSuccess) e = apply_choice(b, best);
    if (e != hipSuccess) return device_fail(e, "autotuning the batch");
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        g_tune_cache[key] = best;
    }
    if (ppl_out) *ppl_out = best.ppl;
    return BSS_OK;
}

bss_status bss_batch_set_member_ppl(bss_batch* b, const int32_t* ppl)
{
    if (!b || !ppl) return fail(BSS_E_INVAL, "batch and ppl must not be NULL");
    if (b->captured) return fail(BSS_E_STATE, "set the particles per lane before capturing");
    if (!plain_batch(b))
        return fail(BSS_E_INVAL, "per-member particles per lane: batches whose members neither "
                                 "repair their samples, redraw their particles nor have "
                                 "half-space constraints");
    std::vector<int> mp(b->n);
    for (int i = 0; i < b->n; ++i) {
        const int P = ppl[i], M = b->ctxs[i]->p.M;
        if (P != 1 && P != 2 && P != 4 && P != 8)
            return fail(BSS_E_INVAL, "member %d: particles per lane must be 1, 2, 4 or 8", i);
        if ((M + P - 1) / P > 64)
            return fail(BSS_E_INVAL, "member %d: M=%d needs more than 64 lanes with %d particles "
                        "per lane", i, M, P);
        mp[i] = P;
    }
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return device_fail(e, "synchronising");
    b->member_ppl = mp;
    e = batch_layout(b, 0, b->split ? 1 : 0);
    if (e != hipSuccess) return device_fail(e, "laying out the batch");
    return BSS_OK;
}

bss_status bss_batch_member_shape(const bss_batch* b, int32_t i, int32_t* lanes, int32_t* ppl)
{
    if (!b) return fail(BSS_E_INVAL, "batch is NULL");
    if (i < 0 || i >= b->n) return fail(BSS_E_INVAL, "member %d of %d", i, b->n);
    if (lanes) *lanes = b->lanes[i];
    if (ppl) *ppl = b->ppls[i];
    return BSS_OK;
}

bss_status bss_batch_set_grid(bss_batch* b, int32_t persistent)
{
    if (!b) return fail(BSS_E_INVAL, "batch is NULL");
    if (persistent != 0 && persistent != 1) return fail(BSS_E_INVAL, "persistent must be 0 or 1");
    if (b->captured) return fail(BSS_E_STATE, "set the grid before capturing the batch");
    if (persistent == 1 && !plain_batch(b))
        return fail(BSS_E_INVAL, "the persistent grid runs batches whose members neither repair "
                                 "their samples, redraw their particles nor have half-space "
                                 "constraints");
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return device_fail(e, "synchronising");
    b->persistent = persistent == 1;
    return BSS_OK;
}

bss_status bss_batch_info(bss_batch* b, int32_t* nblocks, int32_t* ppl, int32_t* split)
{
    if (!b) return fail(BSS_E_INVAL, "batch is NULL");
    if (nblocks) *nblocks = b->nblocks;
    if (ppl) *ppl = b->ppl;
    if (split) *split = (b->split ? 1 : 0) | (b->persistent ? 2 : 0);
    return BSS_OK;
}

void bss_batch_destroy(bss_batch* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    // hand each context its advanced state back (its own launch shape is kept)
    for (int i = 0; i < b->n; ++i) {
        bss_ctx* c = b->ctxs[i];
        int32_t stv[4];
        if (hipMemcpy(stv, (char*)(b->d_desc + i) + kStateOffset, kStateBytes,
                      hipMemcpyDeviceToHost) == hipSuccess) {
            stv[3] = 0;
            (void)hipMemcpy((char*)c->d_desc + kStateOffset, stv, kStateBytes,
                            hipMemcpyHostToDevice);
        }
    }
    batch_free(b);
}

const char* bss_last_error(void) { return last_error_message(); }

// ---- stand-alone kernels -----------------------------------------------------------------------
bss_status bss_dev_philox(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n,
                          void* stream)
{
    if (n < 0 || (n > 0 && (!ctr || !out))) return fail(BSS_E_INVAL, "bad arguments");
    hipError_t e = launch_philox((uint32_t)seed, (uint32_t)(seed >> 32), ctr, out, n,
                                 (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "philox launch");
    return BSS_OK;
}

bss_status bss_dev_normals(uint64_t seed, const uint32_t* ctr, float* z, int64_t n, void* stream)
{
    if (n < 0 || (n > 0 && (!ctr || !z))) return fail(BSS_E_INVAL, "bad arguments");
    hipError_t e = launch_normals((uint32_t)seed, (uint32_t)(seed >> 32), ctr, z, n,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "normals launch");
    return BSS_OK;
}

bss_status bss_dev_disturbance(uint64_t seed, uint32_t solve_index, int32_t K, int32_t M,
                               int32_t T, int32_t crn, int32_t lanes, int32_t ppl, float* w,
                               uint32_t* words, void* stream)
{
    if (K < 0 || M < 0 || T < 0) return fail(BSS_E_INVAL, "K, M, T must be >= 0");
    if (lanes != 8 && lanes != 16 && lanes != 32 && lanes != 64)
        return fail(BSS_E_INVAL, "lanes must be 8, 16, 32 or 64 (got %d)", lanes);
    if (ppl != 1 && ppl != 2 && ppl != 4 && ppl != 8)
        return fail(BSS_E_INVAL, "ppl must be 1, 2, 4 or 8 (got %d)", ppl);
    if ((int64_t)lanes * ppl < M)
        return fail(BSS_E_INVAL, "lanes * ppl = %d holds fewer than M = %d particles",
                    lanes * ppl, M);
    if ((int64_t)K * M * T > 0 && (!w || !words)) return fail(BSS_E_INVAL, "bad arguments");
    hipError_t e = launch_disturbance(lanes, ppl, (uint32_t)seed, (uint32_t)(seed >> 32),
                                      solve_index, K, M, T, crn ? 1 : 0, w, words,
                                      (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "disturbance launch");
    return BSS_OK;
}

bss_status bss_dev_model_step(const bss_params* p, const float* x, const float* u, float* xn,
                              int64_t n, void* stream)
{
    bss_status st = bss_validate(p);
    if (st != BSS_OK) return st;
    if (n < 0 || (n > 0 && (!x || !u || !xn))) return fail(BSS_E_INVAL, "bad arguments");
    hipError_t e = launch_model_step(make_car(*p), x, u, xn, n, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "model_step launch");
    return BSS_OK;
}

bss_status bss_dev_model_step8(const bss_params* p, const float* x, const float* u, float* xn,
                               int64_t n, void* stream)
{
    bss_status st = bss_validate(p);
    if (st != BSS_OK) return st;
    if (p->vehicle != 1) return fail(BSS_E_INVAL, "bss_dev_model_step8 needs vehicle = 1");
    if (n < 0 || (n > 0 && (!x || !u || !xn))) return fail(BSS_E_INVAL, "bad arguments");
    hipError_t e = launch_model_step8(make_car8(*p), x, u, xn, n, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "model_step8 launch");
    return BSS_OK;
}

bss_status bss_dev_sdf(double a, double b, const double* pts, double* out, int64_t n,
                       void* stream)
{
    if (!finite_pos(a) || !finite_pos(b)) return fail(BSS_E_INVAL, "semi-axes must be > 0");
    if (n < 0 || (n > 0 && (!pts || !out))) return fail(BSS_E_INVAL, "bad arguments");
    hipError_t e = launch_sdf(a, b, pts, out, n, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "sdf launch");
    return BSS_OK;
}

bss_status bss_dev_score(const bss_params* p, const double* mom, const float* u, const double* v,
                         double* S, void* stream)
{
    bss_status st = bss_validate(p);
    if (st != BSS_OK) return st;
    if (!mom || !u || !v || !S) return fail(BSS_E_INVAL, "NULL buffer");
    if (p->n_con > 0)
        return fail(BSS_E_INVAL,
                    "the staged score takes no constraint variances (n_con must be 0)");
    hipError_t e = launch_score(p->K, p->T, make_score(*p), mom, u, v, S, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "score launch");
    return BSS_OK;
}

size_t bss_dev_update_workspace(int32_t K, int32_t T)
{
    if (K < 1 || T < 1) return 0;
    return align256((size_t)T * 2 * sizeof(double)) +
           (size_t)partial_blocks(K) * (size_t)partial_stride(T) * sizeof(double);
}

bss_status bss_dev_update(const bss_params* p, const double* S, const float* u, double* v,
                          double* stats, void* workspace, void* stream)
{
    bss_status st = bss_validate(p);
    if (st != BSS_OK) return st;
    if (!S || !u || !v || !stats || !workspace) return fail(BSS_E_INVAL, "NULL buffer");
    hipStream_t s = (hipStream_t)stream;
    double* v_out = (double*)workspace;
    double* partial = (double*)((char*)workspace + align256((size_t)p->T * 2 * sizeof(double)));
    hipError_t e = launch_partials(p->K, p->T, p->lambda, S, u, v, partial, s);
    if (e == hipSuccess)
        e = launch_merge_plain(p->T, partial_blocks(p->K), p->lambda, partial, v, v_out, stats, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(v, v_out, (size_t)p->T * 2 * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return device_fail(e, "update launch");
    return BSS_OK;
}

bss_status bss_dev_repair(const bss_params* p, const double* mom, const double* u_in,
                          double* u_out, int64_t n, void* stream)
{
    bss_status st = bss_validate(p);
    if (st != BSS_OK) return st;
    if (n < 0 || (n > 0 && (!mom || !u_in || !u_out))) return fail(BSS_E_INVAL, "bad arguments");
    if (p->n_con > 0)
        return fail(BSS_E_INVAL,
                    "the staged repair takes no constraint variances (n_con must be 0)");
    hipError_t e = launch_repair(make_score(*p), mom, u_in, u_out, n, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "repair launch");
    return BSS_OK;
}

}  // extern "C"
