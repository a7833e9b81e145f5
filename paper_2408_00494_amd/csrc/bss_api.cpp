// bss_api.cpp -- C ABI of libbssmppi: parameter checks, contexts, device buffers and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/bssmppi.h"
#include "bss_internal.h"

using namespace bss;

namespace {

thread_local std::string g_err;

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
    s.nu = backoff_of(p);
    s.gamma = p.gamma;
    s.lambda = p.lambda;
    s.shield_iters = p.shield_iters;
    s.shield_gmin = p.shield_gmin;
    s.shield_fd = p.shield_fd;
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

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct bss_ctx {
    bss_params p;
    bss_allocator alloc;
    bool has_alloc;
    hipStream_t stream;
    void* block;
    double* vbuf[2];         // ping-pong pair of mean sequences [T][2]
    int cur;                 // index of the current mean sequence
    int pending_shift;       // warm-start shifts not yet applied to vbuf[cur]
    float* u;
    double* mom;
    double* S;
    double* stats;
    double* partial;
    double* x0;
    double* Sigma0;
    double* host;            // pinned [16]
    uint32_t solve_index;
    int32_t outputs;         // BSS_OUT_* flags
    LaunchShape shape;
    bool timing;
    std::vector<hipEvent_t> ev;   // pairs (start, stop)
    size_t ev_used;
};

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
    if (p->shield_iters > 0 && (!finite_pos(p->shield_fd) || !finite_nonneg(p->shield_gmin)))
        return fail(BSS_E_INVAL, "shield_fd must be > 0 and shield_gmin >= 0");
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
    c->shape = choose_shape(p->K, p->M, p->T, p->lanes);
    c->timing = false;
    c->ev_used = 0;
    c->solve_index = 0;

    const size_t K = (size_t)p->K, T = (size_t)p->T;
    const size_t G = (size_t)solve_blocks(p->K, 8);   // most blocks any launch shape uses
    const size_t sz_v = align256(T * 2 * sizeof(double));
    const size_t sz_u = align256(K * T * 2 * sizeof(float));
    const size_t sz_mom = align256(K * (T + 1) * 9 * sizeof(double));
    const size_t sz_S = align256(K * sizeof(double));
    const size_t sz_stats = align256(8 * sizeof(double));
    const size_t sz_part = align256(G * (2 * T + 4) * sizeof(double));
    const size_t sz_x0 = 256;
    const size_t sz_sig = align256(36 * sizeof(double));
    const size_t total = 2 * sz_v + sz_u + sz_mom + sz_S + sz_stats + sz_part + sz_x0 + sz_sig;

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
    c->vbuf[0] = (double*)b;
    b += sz_v;
    c->vbuf[1] = (double*)b;
    b += sz_v;
    c->u = (float*)b;
    b += sz_u;
    c->mom = (double*)b;
    b += sz_mom;
    c->S = (double*)b;
    b += sz_S;
    c->stats = (double*)b;
    b += sz_stats;
    c->partial = (double*)b;
    b += sz_part;
    c->x0 = (double*)b;
    b += sz_x0;
    c->Sigma0 = (double*)b;
    c->cur = 0;
    c->pending_shift = 0;
    c->outputs = BSS_OUT_CONTROLS;

    hipError_t e = hipHostMalloc((void**)&c->host, 16 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        if (c->has_alloc) c->alloc.release(block, c->alloc.user);
        else (void)hipFree(block);
        delete c;
        return fail(BSS_E_NOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    // zero the warm start and stats (whole block: also makes unused slots defined)
    e = hipMemsetAsync(block, 0, total, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
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

static bss_status enqueue_solve(bss_ctx* c, const double* x0_dev, const double* Sigma0_dev)
{
    const bss_params& p = c->p;
    SolveArgs a;
    a.K = p.K;
    a.M = p.M;
    a.T = p.T;
    a.vshift = c->pending_shift;
    a.solve_index = c->solve_index;
    a.key0 = (uint32_t)p.seed;
    a.key1 = (uint32_t)(p.seed >> 32);
    a.steer_max = (float)p.steer_max;
    a.accel_max = (float)p.accel_max;
    a.sig_eps0 = (float)p.sigma_eps[0];
    a.sig_eps1 = (float)p.sigma_eps[1];
    a.sig_w0 = (float)p.sigma_w[0];
    a.sig_w1 = (float)p.sigma_w[1];
    a.sig_w2 = (float)p.sigma_w[2];
    a.car = make_car(p);
    a.sc = make_score(p);
    a.x0 = x0_dev;
    a.Sigma0 = Sigma0_dev;
    a.v = c->vbuf[c->cur];
    a.u = (c->outputs & BSS_OUT_CONTROLS) ? c->u : nullptr;
    a.mom = c->mom;
    a.S = c->S;
    a.partial = c->partial;

    hipError_t e;
    if (c->timing) {
        if (c->ev_used + 2 > c->ev.size()) {
            for (int i = 0; i < 64; ++i) {
                hipEvent_t ev;
                e = hipEventCreate(&ev);
                if (e != hipSuccess) return device_fail(e, "hipEventCreate");
                c->ev.push_back(ev);
            }
        }
        e = hipEventRecord(c->ev[c->ev_used], c->stream);
        if (e != hipSuccess) return device_fail(e, "hipEventRecord");
    }
    e = launch_solve(a, c->shape, c->stream);
    if (e != hipSuccess) return device_fail(e, "solve launch");
    if (c->timing) {
        e = hipEventRecord(c->ev[c->ev_used + 1], c->stream);
        if (e != hipSuccess) return device_fail(e, "hipEventRecord");
        c->ev_used += 2;
    }
    MergeArgs ma;
    ma.T = p.T;
    ma.G = solve_blocks(p.K, c->shape.lanes);
    ma.vshift = c->pending_shift;
    ma.lambda = p.lambda;
    ma.partial = c->partial;
    ma.v_in = c->vbuf[c->cur];
    ma.v_out = c->vbuf[1 - c->cur];
    ma.stats = c->stats;
    e = launch_merge(ma, c->stream);
    if (e != hipSuccess) return device_fail(e, "merge launch");
    c->cur = 1 - c->cur;
    c->pending_shift = 0;
    c->solve_index += 1;
    return BSS_OK;
}

bss_status bss_solve_async(bss_ctx* c, const double* x0_dev, const double* Sigma0_dev)
{
    if (!c) return fail(BSS_E_INVAL, "ctx is NULL");
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
    info->lanes = c->shape.lanes;
    info->ppl = c->shape.ppl;
}

bss_status bss_solve(bss_ctx* c, const double x0[6], const double* Sigma0, double u0_out[2],
                     bss_info* info)
{
    if (!c) return fail(BSS_E_INVAL, "ctx is NULL");
    if (!x0 || !u0_out) return fail(BSS_E_INVAL, "x0 and u0_out must not be NULL");
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(x0[i])) return fail(BSS_E_INVAL, "x0[%d] is not finite", i);
    if (Sigma0) {
        for (int i = 0; i < 36; ++i)
            if (!std::isfinite(Sigma0[i])) return fail(BSS_E_INVAL, "Sigma0[%d] not finite", i);
        for (int i = 0; i < 6; ++i)
            if (Sigma0[i * 6 + i] < 0.0) return fail(BSS_E_INVAL, "Sigma0 has a negative variance");
    }
    hipError_t e = hipMemcpyAsync(c->x0, x0, 6 * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && Sigma0)
        e = hipMemcpyAsync(c->Sigma0, Sigma0, 36 * sizeof(double), hipMemcpyHostToDevice,
                           c->stream);
    if (e != hipSuccess) return device_fail(e, "staging x0");
    bss_status st = enqueue_solve(c, c->x0, Sigma0 ? c->Sigma0 : nullptr);
    if (st != BSS_OK) return st;
    e = hipMemcpyAsync(c->host, c->stats, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
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
    if (!c) return fail(BSS_E_INVAL, "ctx is NULL");
    if (c->pending_shift < c->p.T - 1) c->pending_shift += 1;
    return BSS_OK;
}

bss_status bss_set_outputs(bss_ctx* c, int32_t flags)
{
    if (!c) return fail(BSS_E_INVAL, "ctx is NULL");
    if (flags & ~BSS_OUT_CONTROLS) return fail(BSS_E_INVAL, "unknown flags");
    c->outputs = flags;
    return BSS_OK;
}

bss_status bss_get_buffers(const bss_ctx* c, bss_buffers* out)
{
    if (!c || !out) return fail(BSS_E_INVAL, "NULL argument");
    out->v = c->vbuf[c->cur];
    out->u = c->u;
    out->mom = c->mom;
    out->S = c->S;
    out->stats = c->stats;
    out->x0 = c->x0;
    out->Sigma0 = c->Sigma0;
    out->v_shift = c->pending_shift;
    return BSS_OK;
}

bss_status bss_get_controls(bss_ctx* c, double* v_host)
{
    if (!c || !v_host) return fail(BSS_E_INVAL, "NULL argument");
    const int T = c->p.T;
    std::vector<double> tmp((size_t)T * 2);
    hipError_t e = hipMemcpyAsync(tmp.data(), c->vbuf[c->cur], (size_t)T * 2 * sizeof(double),
                                  hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_fail(e, "reading controls");
    for (int t = 0; t < T; ++t) {
        const int r = t + c->pending_shift < T ? t + c->pending_shift : T - 1;
        v_host[2 * t] = tmp[2 * r];
        v_host[2 * t + 1] = tmp[2 * r + 1];
    }
    return BSS_OK;
}

bss_status bss_set_controls(bss_ctx* c, const double* v_host)
{
    if (!c || !v_host) return fail(BSS_E_INVAL, "NULL argument");
    for (int i = 0; i < 2 * c->p.T; ++i)
        if (!std::isfinite(v_host[i])) return fail(BSS_E_INVAL, "controls must be finite");
    hipError_t e = hipMemcpyAsync(c->vbuf[c->cur], v_host, (size_t)c->p.T * 2 * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_fail(e, "writing controls");
    c->pending_shift = 0;
    return BSS_OK;
}

bss_status bss_set_solve_index(bss_ctx* c, uint32_t s)
{
    if (!c) return fail(BSS_E_INVAL, "ctx is NULL");
    c->solve_index = s;
    return BSS_OK;
}

bss_status bss_get_solve_index(const bss_ctx* c, uint32_t* s)
{
    if (!c || !s) return fail(BSS_E_INVAL, "NULL argument");
    *s = c->solve_index;
    return BSS_OK;
}

bss_status bss_get_info(bss_ctx* c, bss_info* info)
{
    if (!c || !info) return fail(BSS_E_INVAL, "NULL argument");
    hipError_t e = hipMemcpyAsync(c->host, c->stats, 8 * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
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

bss_status bss_set_lanes(bss_ctx* c, int32_t lanes)
{
    if (!c) return fail(BSS_E_INVAL, "ctx is NULL");
    bss_params q = c->p;
    q.lanes = lanes;
    bss_status st = bss_validate(&q);
    if (st != BSS_OK) return st;
    c->shape = choose_shape(q.K, q.M, q.T, lanes);
    return BSS_OK;
}

void bss_destroy(bss_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t ev : c->ev) (void)hipEventDestroy(ev);
    if (c->block) {
        if (c->has_alloc) c->alloc.release(c->block, c->alloc.user);
        else (void)hipFree(c->block);
    }
    if (c->host) (void)hipHostFree(c->host);
    delete c;
}

const char* bss_last_error(void) { return g_err.c_str(); }

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
    SolveArgs a;
    std::memset(&a, 0, sizeof(a));
    a.K = p->K;
    a.M = p->M;
    a.T = p->T;
    a.vshift = 0;
    a.sc = make_score(*p);
    a.mom = const_cast<double*>(mom);
    a.u = const_cast<float*>(u);
    a.v = v;
    a.S = S;
    hipError_t e = launch_score(a, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "score launch");
    return BSS_OK;
}

size_t bss_dev_update_workspace(int32_t K, int32_t T)
{
    if (K < 1 || T < 1) return 0;
    return align256((size_t)T * 2 * sizeof(double)) +
           (size_t)partial_blocks(K) * (2 * (size_t)T + 4) * sizeof(double);
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
    if (e != hipSuccess) return device_fail(e, "partial launch");
    MergeArgs ma;
    ma.T = p->T;
    ma.G = partial_blocks(p->K);
    ma.vshift = 0;
    ma.lambda = p->lambda;
    ma.partial = partial;
    ma.v_in = v;
    ma.v_out = v_out;
    ma.stats = stats;
    e = launch_merge(ma, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(v, v_out, (size_t)p->T * 2 * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return device_fail(e, "merge launch");
    return BSS_OK;
}

bss_status bss_dev_repair(const bss_params* p, const double* mom, const double* u_in,
                          double* u_out, int64_t n, void* stream)
{
    bss_status st = bss_validate(p);
    if (st != BSS_OK) return st;
    if (n < 0 || (n > 0 && (!mom || !u_in || !u_out))) return fail(BSS_E_INVAL, "bad arguments");
    hipError_t e = launch_repair(make_score(*p), mom, u_in, u_out, n, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "repair launch");
    return BSS_OK;
}

}  // extern "C"
