// bss_server.cpp -- serving runtime of libbssmppi: many vehicles, each running the receding-horizon
// loop of Alg. 1 with its own track, noise and warm start, whose solve requests are batched as
// they arrive.
//
// Resident per vehicle (device): the ping-pong pair of mean control sequences.  Tracked per
// vehicle on the host: which buffer is current, the pending warm-start shift and the solve index
// (the Philox counter word of its next solve); the device advances the same fields in the
// launch's descriptor, and the host mirrors them when it launches, so nothing is read back.
//
// Scratch (belief records, costs, block partials) belongs to in-flight solves only: each of the
// n_streams slots owns an arena of hbm_budget / n_streams bytes, and a request is admitted into a
// batch while its scratch fits in the slot's arena.  Whenever a slot is free, every admissible
// pending request (oldest first, one per vehicle: a vehicle's next solve needs the result of its
// previous one) goes out as one solve launch and one merge launch on that slot's stream, so
// requests that arrive while others are on the GPU overlap with them on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <new>
#include <vector>

#include "../../include/bssmppi.h"
#include "bss_host.h"
#include "bss_internal.h"

using namespace bss;

namespace {

struct Request {
    int64_t id;
    int32_t vehicle, K, M;
    double nu;
    double x0[6];
};

struct Vehicle {
    bss_params p;
    InstanceDesc base;       // static fields of the vehicle's problem
    double* v[2];            // device ping-pong pair [T][2]
    int32_t cur, vshift;
    uint32_t solve_index;
    bool busy;               // a solve of this vehicle is in flight
    int64_t pending;         // requests submitted and not yet completed
};

struct Slot {
    hipStream_t stream;
    hipEvent_t done;
    char* d_region;          // descriptors | blocks | merge columns | states (device)
    char* h_region;          // pinned staging of the same
    size_t region_bytes;
    double* d_stats;         // [max_batch][8]
    double* h_stats;         // pinned copy of the stats of the batch in flight
    char* arena;
    size_t arena_bytes;
    bool busy;
    std::vector<int64_t> reqs;
    std::vector<int32_t> vehicles;
};

double now_s()
{
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

size_t scratch_bytes(int K, int T, int lanes)
{
    const size_t blocks = (size_t)solve_blocks(K, lanes);
    return align256((size_t)K * (T + 1) * 9 * sizeof(double)) +
           align256((size_t)K * sizeof(double)) +
           align256(blocks * (size_t)partial_stride(T) * sizeof(double));
}

}  // namespace

struct bss_server {
    bss_server_config cfg;
    int ppl;
    std::vector<Vehicle> veh;
    std::vector<Slot> slots;
    double* d_vbuf;          // every vehicle's pair of mean sequences
    std::deque<Request> pending;
    std::deque<bss_completion> completed;
    int64_t next_id;
    size_t max_blocks;
    // per-launch host scratch (reused)
    std::vector<InstanceDesc> descs;
    std::vector<BlockDesc> blocks;
    std::vector<MergeDesc> cols;
    std::vector<char> seen;
};

namespace {

void server_free(bss_server* s)
{
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.d_region) (void)hipFree(sl.d_region);
        if (sl.h_region) (void)hipHostFree(sl.h_region);
        if (sl.d_stats) (void)hipFree(sl.d_stats);
        if (sl.h_stats) (void)hipHostFree(sl.h_stats);
        if (sl.arena) (void)hipFree(sl.arena);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (s->d_vbuf) (void)hipFree(s->d_vbuf);
    delete s;
}

// Retire every slot whose batch has completed.
bss_status retire(bss_server* s, int* n_retired)
{
    *n_retired = 0;
    for (Slot& sl : s->slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return device_fail(q, "batch completion");
        const double t = now_s();
        for (size_t i = 0; i < sl.reqs.size(); ++i) {
            const double* st = sl.h_stats + 8 * i;
            bss_completion c;
            c.req = sl.reqs[i];
            c.vehicle = sl.vehicles[i];
            c.status = st[4] != 0.0 ? BSS_E_NUMERIC : BSS_OK;
            c.u0[0] = st[5];
            c.u0[1] = st[6];
            c.t_done = t;
            s->completed.push_back(c);
            Vehicle& v = s->veh[c.vehicle];
            v.busy = false;
            v.pending -= 1;
        }
        sl.reqs.clear();
        sl.vehicles.clear();
        sl.busy = false;
        ++*n_retired;
    }
    return BSS_OK;
}

// Form one batch from the pending requests and launch it on a free slot.  Returns BSS_OK with
// *launched = 0 when nothing is admissible.
bss_status launch_batch(bss_server* s, Slot& sl, int* launched)
{
    *launched = 0;
    const int T = s->cfg.T;
    const int maxb = s->cfg.max_batch;
    std::vector<InstanceDesc>& descs = s->descs;
    std::vector<BlockDesc>& blocks = s->blocks;
    std::vector<MergeDesc>& cols = s->cols;
    descs.clear();
    blocks.clear();
    cols.clear();
    std::fill(s->seen.begin(), s->seen.end(), 0);
    sl.reqs.clear();
    sl.vehicles.clear();
    std::vector<double> x0s;
    size_t used = 0, lds = 0;
    bool shield = false, ring_fits = true, resample = false, con = false;
    // pick requests oldest first; skip a vehicle already in flight or already seen in this scan
    std::deque<Request>& pend = s->pending;
    std::vector<size_t> taken;
    for (size_t qi = 0; qi < pend.size() && (int)descs.size() < maxb; ++qi) {
        const Request& r = pend[qi];
        Vehicle& v = s->veh[r.vehicle];
        if (s->seen[r.vehicle] || v.busy) {
            s->seen[r.vehicle] = 1;
            continue;
        }
        s->seen[r.vehicle] = 1;
        const LaunchShape sh = choose_shape(r.K, r.M, T, 0, s->ppl, 0);
        const size_t con_bytes =
            align256((size_t)r.K * (T + 1) * (size_t)v.p.n_con * sizeof(double));
        const size_t base_bytes = scratch_bytes(r.K, T, sh.lanes);
        const size_t need = base_bytes + con_bytes;   // beliefs, costs, partials | variances
        if (used + need > sl.arena_bytes) continue;   // waits for memory (admission)
        const int nb = solve_blocks(r.K, sh.lanes);
        if (blocks.size() + (size_t)nb > s->max_blocks) continue;
        const int i = (int)descs.size();
        InstanceDesc d = v.base;
        d.K = r.K;
        d.M = r.M;
        d.lanes = sh.lanes;
        d.ppl = s->ppl;
        d.nblocks = nb;
        d.x0_index = i;
        d.cur = v.cur;
        d.vshift = v.vshift;
        d.solve_index = v.solve_index;
        d.done = 0;
        d.shift_after = 1;
        d.status = 0;
        d.sc.nu = r.nu;
        d.v[0] = v.v[0];
        d.v[1] = v.v[1];
        d.u = nullptr;
        char* a = sl.arena + used;
        d.mom = (double*)a;
        a += align256((size_t)r.K * (T + 1) * 9 * sizeof(double));
        d.S = (double*)a;
        a += align256((size_t)r.K * sizeof(double));
        d.partial = (double*)a;
        d.cvar = v.p.n_con > 0 ? (double*)(sl.arena + used + base_bytes) : nullptr;
        d.stats = sl.d_stats + 8 * i;
        used += need;
        shield = shield || v.p.shield_iters > 0;
        resample = resample || v.p.belief != 0;
        con = con || v.p.n_con > 0;
        descs.push_back(d);
        append_blocks(blocks, i, r.K, sh.lanes);
        for (int c = 0; c < 2 * T; ++c) cols.push_back(MergeDesc{i, c});
        x0s.insert(x0s.end(), r.x0, r.x0 + 6);
        sl.reqs.push_back(r.id);
        sl.vehicles.push_back(r.vehicle);
        taken.push_back(qi);
    }
    if (descs.empty()) return BSS_OK;
    // the launch's variant holds the constraint rows of the moment exchange when any member has
    // constraints
    for (const InstanceDesc& d : descs) {
        lds = std::max(lds, solve_lds_bytes(d.lanes, T, s->ppl, false, false, con));
        ring_fits = ring_fits && solve_base_lds_bytes(d.lanes, T, s->ppl, true) <= kMaxLds &&
                    split_fits(d.lanes, T, s->ppl, false, con, kStaticLdsSlots);
    }
    // a batch too small to put two waves on every SIMD generates its noise in separate waves
    const bool split = !shield && !resample && ring_fits && (int64_t)blocks.size() * 4 < 2 * 1024;
    if (split) {
        size_t l2 = 0;
        for (const InstanceDesc& d : descs)
            l2 = std::max(l2, solve_lds_bytes(d.lanes, T, s->ppl, true, false, con));
        lds = l2;
    }

    // pack descriptors | blocks | columns | states into the slot's pinned staging, one upload
    const size_t o_desc = 0;
    const size_t o_blk = align256(o_desc + descs.size() * sizeof(InstanceDesc));
    const size_t o_col = align256(o_blk + blocks.size() * sizeof(BlockDesc));
    const size_t o_x0 = align256(o_col + cols.size() * sizeof(MergeDesc));
    const size_t total = o_x0 + x0s.size() * sizeof(double);
    if (total > sl.region_bytes) return fail(BSS_E_STATE, "batch staging overflow");
    std::memcpy(sl.h_region + o_desc, descs.data(), descs.size() * sizeof(InstanceDesc));
    std::memcpy(sl.h_region + o_blk, blocks.data(), blocks.size() * sizeof(BlockDesc));
    std::memcpy(sl.h_region + o_col, cols.data(), cols.size() * sizeof(MergeDesc));
    std::memcpy(sl.h_region + o_x0, x0s.data(), x0s.size() * sizeof(double));
    hipError_t e = hipMemcpyAsync(sl.d_region, sl.h_region, total, hipMemcpyHostToDevice,
                                  sl.stream);
    const InstanceDesc* d_desc = (const InstanceDesc*)(sl.d_region + o_desc);
    if (e == hipSuccess)
        e = launch_solve(d_desc, (const BlockDesc*)(sl.d_region + o_blk), (int)blocks.size(),
                         s->ppl, shield, split, resample, con, lds,
                         (const double*)(sl.d_region + o_x0), nullptr, 0, sl.stream);
    if (e == hipSuccess)
        e = launch_merge(d_desc, (const MergeDesc*)(sl.d_region + o_col), (int)cols.size(), 0,
                         sl.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sl.h_stats, sl.d_stats, descs.size() * 8 * sizeof(double),
                           hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    if (e != hipSuccess) return device_fail(e, "batch launch");

    // the device advances each descriptor exactly like this
    for (size_t i = 0; i < descs.size(); ++i) {
        Vehicle& v = s->veh[sl.vehicles[i]];
        v.busy = true;
        v.cur = 1 - v.cur;
        v.vshift = 1;
        v.solve_index += 1u;
    }
    for (size_t t = taken.size(); t-- > 0;) pend.erase(pend.begin() + (std::ptrdiff_t)taken[t]);
    sl.busy = true;
    *launched = (int)descs.size();
    return BSS_OK;
}

bss_status vehicle_idle(const bss_server* s, int32_t vehicle)
{
    if (!s) return fail(BSS_E_INVAL, "server is NULL");
    if (vehicle < 0 || vehicle >= s->cfg.n_vehicles)
        return fail(BSS_E_INVAL, "vehicle %d out of range", vehicle);
    if (s->veh[vehicle].busy || s->veh[vehicle].pending > 0)
        return fail(BSS_E_STATE, "vehicle %d has requests pending or in flight", vehicle);
    return BSS_OK;
}

}  // namespace

extern "C" {

void bss_server_config_default(bss_server_config* c)
{
    if (!c) return;
    c->n_vehicles = 256;
    c->T = 50;
    c->K_max = 8192;
    c->M_max = 128;
    c->ppl = 4;
    c->n_streams = 2;
    c->max_batch = 256;
    c->hbm_budget = (uint64_t)32 << 30;
}

bss_status bss_server_create(const bss_server_config* cfg, const bss_params* vehicles,
                             bss_server** out)
{
    if (!out) return fail(BSS_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!cfg || !vehicles) return fail(BSS_E_INVAL, "config and vehicle parameters are required");
    const bss_server_config& c = *cfg;
    if (c.n_vehicles < 1 || c.n_vehicles > (1 << 20)) return fail(BSS_E_INVAL, "n_vehicles");
    if (c.T < 1 || c.T > kMaxT) return fail(BSS_E_INVAL, "T must be in [1, %d]", kMaxT);
    if (c.K_max < 1 || c.K_max > (1 << 20)) return fail(BSS_E_INVAL, "K_max must be in [1, 2^20]");
    if (c.M_max < 1 || c.M_max > 512) return fail(BSS_E_INVAL, "M_max must be in [1, 512]");
    const int ppl = c.ppl == 0 ? 4 : c.ppl;
    if (ppl != 1 && ppl != 2 && ppl != 4 && ppl != 8) return fail(BSS_E_INVAL, "ppl");
    if ((c.M_max + ppl - 1) / ppl > 64)
        return fail(BSS_E_INVAL, "M_max=%d needs more than 64 lanes with %d particles per lane",
                    c.M_max, ppl);
    if (c.n_streams < 1 || c.n_streams > 16) return fail(BSS_E_INVAL, "n_streams must be 1..16");
    if (c.max_batch < 1 || c.max_batch > 4096)
        return fail(BSS_E_INVAL, "max_batch must be 1..4096");
    int max_con = 0;
    for (int i = 0; i < c.n_vehicles; ++i) {
        bss_params q = vehicles[i];
        q.K = c.K_max;
        q.M = c.M_max;
        q.T = c.T;
        bss_status st = bss_validate(&q);
        if (st != BSS_OK) return st;
        if (q.local_repair != 0)
            return fail(BSS_E_INVAL, "vehicle %d: the repair of the update (local_repair) runs per "
                        "context, not in the server's batched launches", i);
        if (q.vehicle != 0)
            return fail(BSS_E_INVAL, "vehicle %d: the 8-state vehicle model (vehicle = 1) runs "
                        "per context, not in the server's batched launches", i);
        max_con = std::max(max_con, (int)q.n_con);
    }
    // one request of K_max per stream must fit, with the variances of the most constrained vehicle
    size_t worst = 0;
    for (int lanes = 8; lanes <= 64; lanes *= 2)
        worst = std::max(worst, scratch_bytes(c.K_max, c.T, lanes));
    worst += align256((size_t)c.K_max * (c.T + 1) * (size_t)max_con * sizeof(double));
    if (c.hbm_budget / (uint64_t)c.n_streams < worst)
        return fail(BSS_E_INVAL, "hbm_budget %llu is below n_streams x %zu bytes (one request of "
                    "K_max per stream)", (unsigned long long)c.hbm_budget, worst);

    bss_server* s = new (std::nothrow) bss_server();
    if (!s) return fail(BSS_E_NOMEM, "host allocation failed");
    s->cfg = c;
    s->ppl = ppl;
    s->next_id = 0;
    s->d_vbuf = nullptr;
    s->max_blocks = (size_t)c.max_batch * (size_t)solve_blocks(c.K_max, 64);
    s->seen.assign((size_t)c.n_vehicles, 0);
    const size_t vbytes = (size_t)c.T * 2 * sizeof(double);
    hipError_t e = hipMalloc((void**)&s->d_vbuf, 2 * vbytes * (size_t)c.n_vehicles);
    if (e != hipSuccess) {
        s->d_vbuf = nullptr;
        server_free(s);
        return fail(BSS_E_NOMEM, "vehicle state: %s", hipGetErrorString(e));
    }
    e = hipMemset(s->d_vbuf, 0, 2 * vbytes * (size_t)c.n_vehicles);
    s->veh.resize((size_t)c.n_vehicles);
    for (int i = 0; i < c.n_vehicles; ++i) {
        Vehicle& v = s->veh[i];
        v.p = vehicles[i];
        v.p.T = c.T;
        v.base = make_desc(v.p);
        v.v[0] = s->d_vbuf + (size_t)i * 2 * c.T * 2;
        v.v[1] = v.v[0] + (size_t)c.T * 2;
        v.cur = 0;
        v.vshift = 0;
        v.solve_index = 0;
        v.busy = false;
        v.pending = 0;
    }
    const size_t region = align256((size_t)c.max_batch * sizeof(InstanceDesc)) +
                          align256(s->max_blocks * sizeof(BlockDesc)) +
                          align256((size_t)c.max_batch * 2 * c.T * sizeof(MergeDesc)) +
                          align256((size_t)c.max_batch * 6 * sizeof(double));
    const size_t arena = (size_t)(c.hbm_budget / (uint64_t)c.n_streams) & ~(size_t)255;
    s->slots.resize((size_t)c.n_streams);
    for (Slot& sl : s->slots) {
        sl = Slot{};
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc((void**)&sl.d_region, region);
        if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_region, region, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipMalloc((void**)&sl.d_stats, (size_t)c.max_batch * 8 * sizeof(double));
        if (e == hipSuccess)
            e = hipHostMalloc((void**)&sl.h_stats, (size_t)c.max_batch * 8 * sizeof(double),
                              hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc((void**)&sl.arena, arena);
        sl.region_bytes = region;
        sl.arena_bytes = arena;
        if (e != hipSuccess) break;
    }
    if (e != hipSuccess) {
        server_free(s);
        return fail(BSS_E_NOMEM, "server buffers: %s", hipGetErrorString(e));
    }
    *out = s;
    return BSS_OK;
}

bss_status bss_server_submit(bss_server* s, int32_t vehicle, int32_t K, int32_t M, double delta,
                             const double x0[6], int64_t* req_id)
{
    if (!s || !x0) return fail(BSS_E_INVAL, "NULL argument");
    if (vehicle < 0 || vehicle >= s->cfg.n_vehicles)
        return fail(BSS_E_INVAL, "vehicle %d out of range", vehicle);
    if (K < 1 || K > s->cfg.K_max) return fail(BSS_E_INVAL, "K=%d outside [1, K_max]", K);
    if (M < 1 || M > s->cfg.M_max) return fail(BSS_E_INVAL, "M=%d outside [1, M_max]", M);
    if (s->veh[vehicle].p.belief == 2 && M != 12)
        return fail(BSS_E_INVAL, "vehicle %d uses the sigma-point belief, which has M = 12 "
                    "points (got M=%d)", vehicle, M);
    if (!(delta > 0.0 && delta < 0.5)) return fail(BSS_E_INVAL, "delta must be in (0, 0.5)");
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(x0[i])) return fail(BSS_E_INVAL, "x0[%d] is not finite", i);
    Request r;
    r.id = s->next_id++;
    r.vehicle = vehicle;
    r.K = K;
    r.M = M;
    bss_params q = s->veh[vehicle].p;
    q.delta = delta;
    r.nu = backoff_of(q);
    std::memcpy(r.x0, x0, sizeof(r.x0));
    s->pending.push_back(r);
    s->veh[vehicle].pending += 1;
    if (req_id) *req_id = r.id;
    return BSS_OK;
}

bss_status bss_server_pump(bss_server* s, int32_t* n_launched)
{
    if (!s) return fail(BSS_E_INVAL, "server is NULL");
    int retired = 0, launched_total = 0;
    bss_status st = retire(s, &retired);
    if (st != BSS_OK) return st;
    for (Slot& sl : s->slots) {
        if (sl.busy || s->pending.empty()) continue;
        int launched = 0;
        st = launch_batch(s, sl, &launched);
        if (st != BSS_OK) return st;
        launched_total += launched;
        if (launched == 0) break;   // nothing admissible right now
    }
    if (n_launched) *n_launched = launched_total;
    return BSS_OK;
}

int32_t bss_server_poll(bss_server* s, bss_completion* out, int32_t max)
{
    if (!s || !out || max <= 0) return 0;
    int32_t n = 0;
    while (n < max && !s->completed.empty()) {
        out[n++] = s->completed.front();
        s->completed.pop_front();
    }
    return n;
}

bss_status bss_server_drain(bss_server* s)
{
    if (!s) return fail(BSS_E_INVAL, "server is NULL");
    for (;;) {
        bss_status st = bss_server_pump(s, nullptr);
        if (st != BSS_OK) return st;
        bool busy = !s->pending.empty();
        for (const Slot& sl : s->slots) busy = busy || sl.busy;
        if (!busy) return BSS_OK;
    }
}

bss_status bss_server_get_controls(bss_server* s, int32_t vehicle, double* v_host)
{
    bss_status st = vehicle_idle(s, vehicle);
    if (st != BSS_OK) return st;
    if (!v_host) return fail(BSS_E_INVAL, "NULL argument");
    const Vehicle& v = s->veh[vehicle];
    const int T = s->cfg.T;
    std::vector<double> tmp((size_t)T * 2);
    hipError_t e = hipMemcpy(tmp.data(), v.v[v.cur], tmp.size() * sizeof(double),
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_fail(e, "reading controls");
    for (int t = 0; t < T; ++t) {
        const int r = t + v.vshift < T ? t + v.vshift : T - 1;
        v_host[2 * t] = tmp[2 * r];
        v_host[2 * t + 1] = tmp[2 * r + 1];
    }
    return BSS_OK;
}

bss_status bss_server_set_controls(bss_server* s, int32_t vehicle, const double* v_host)
{
    bss_status st = vehicle_idle(s, vehicle);
    if (st != BSS_OK) return st;
    if (!v_host) return fail(BSS_E_INVAL, "NULL argument");
    for (int i = 0; i < 2 * s->cfg.T; ++i)
        if (!std::isfinite(v_host[i])) return fail(BSS_E_INVAL, "controls must be finite");
    Vehicle& v = s->veh[vehicle];
    hipError_t e = hipMemcpy(v.v[v.cur], v_host, (size_t)s->cfg.T * 2 * sizeof(double),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return device_fail(e, "writing controls");
    v.vshift = 0;
    return BSS_OK;
}

bss_status bss_server_vehicle_state(const bss_server* s, int32_t vehicle, uint32_t* solve_index,
                                    int64_t* pending)
{
    if (!s) return fail(BSS_E_INVAL, "server is NULL");
    if (vehicle < 0 || vehicle >= s->cfg.n_vehicles)
        return fail(BSS_E_INVAL, "vehicle %d out of range", vehicle);
    if (solve_index) *solve_index = s->veh[vehicle].solve_index;
    if (pending) *pending = s->veh[vehicle].pending;
    return BSS_OK;
}

bss_status bss_server_replay(bss_server* s, int64_t n, const double* t_arrival,
                             const int32_t* vehicle, const int32_t* K, const int32_t* M,
                             const double* delta, const double* x0, double* latency_s,
                             double* u0_out, int32_t* status_out)
{
    if (!s || n < 0 || (n > 0 && (!t_arrival || !vehicle || !K || !M || !delta || !x0 ||
                                  !latency_s)))
        return fail(BSS_E_INVAL, "NULL argument");
    for (int64_t i = 0; i < n; ++i) {
        if (i > 0 && !(t_arrival[i] >= t_arrival[i - 1]))
            return fail(BSS_E_INVAL, "arrival times must be non-decreasing");
        if (vehicle[i] < 0 || vehicle[i] >= s->cfg.n_vehicles || K[i] < 1 || K[i] > s->cfg.K_max ||
            M[i] < 1 || M[i] > s->cfg.M_max || !(delta[i] > 0.0 && delta[i] < 0.5))
            return fail(BSS_E_INVAL, "request %lld is out of range", (long long)i);
    }
    bss_status st = bss_server_drain(s);
    if (st != BSS_OK) return st;
    s->completed.clear();
    const int64_t first = s->next_id;
    const double t0 = now_s();
    int64_t next = 0, done = 0;
    std::vector<bss_completion> buf(256);
    while (done < n) {
        const double t = now_s() - t0;
        while (next < n && t_arrival[next] <= t) {
            st = bss_server_submit(s, vehicle[next], K[next], M[next], delta[next], x0 + 6 * next,
                                   nullptr);
            if (st != BSS_OK) return st;
            ++next;
        }
        st = bss_server_pump(s, nullptr);
        if (st != BSS_OK) return st;
        for (;;) {
            const int32_t got = bss_server_poll(s, buf.data(), (int32_t)buf.size());
            for (int32_t j = 0; j < got; ++j) {
                const int64_t i = buf[j].req - first;
                latency_s[i] = buf[j].t_done - (t0 + t_arrival[i]);
                if (u0_out) {
                    u0_out[2 * i] = buf[j].u0[0];
                    u0_out[2 * i + 1] = buf[j].u0[1];
                }
                if (status_out) status_out[i] = buf[j].status;
            }
            done += got;
            if (got < (int32_t)buf.size()) break;
        }
    }
    return BSS_OK;
}

void bss_server_destroy(bss_server* s)
{
    if (!s) return;
    server_free(s);
}

}  // extern "C"
