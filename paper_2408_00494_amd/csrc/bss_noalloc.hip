// bss_noalloc.hip -- one solve without any device allocation, for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// Every scratch buffer of the solve (its descriptor, solve and merge grids, belief records,
// constraint variances, costs and block partials) lives in one file-scope device array of
// kNoAllocScratchBytes that each GPU the library runs on holds until the process ends.  The
// descriptor and the grids are written into it by a set-up kernel that takes the descriptor by
// value, so a call enqueues three kernels and no copy, allocation or synchronisation; calls that
// overlap on one GPU share the array and race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "../../include/bssmppi.h"
#include "bss_host.h"
#include "bss_internal.h"

namespace bss {

namespace {

constexpr size_t kNoAllocScratchBytes = BSS_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// device address of `scratch` on each GPU (the host-side name is only a stand-in), found once
// per device with that device current
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_on_current_device(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Writes the descriptor (state fields included: done = 0 for the merge's counter) and the solve
// and merge grids of one instance into the scratch array.
__global__ __launch_bounds__(256) void setup_kernel(InstanceDesc d, InstanceDesc* dst,
                                                    BlockDesc* blocks, int nblocks, int groups,
                                                    MergeDesc* cols, int ncols)
{
    const int tid = (int)threadIdx.x;
    if (tid == 0) *dst = d;
    for (int b = tid; b < nblocks; b += (int)blockDim.x) blocks[b] = BlockDesc{0, b * groups};
    for (int c = tid; c < ncols; c += (int)blockDim.x) cols[c] = MergeDesc{0, c};
}

struct ScratchLayout {
    size_t desc, blocks, cols, mom, cvar, S, partial, total;
};

ScratchLayout layout_of(const bss_params& p, int nblocks)
{
    const size_t K = (size_t)p.K, T = (size_t)p.T;
    ScratchLayout L;
    size_t o = 0;
    L.desc = o;
    o += align256(sizeof(InstanceDesc));
    L.blocks = o;
    o += align256((size_t)nblocks * sizeof(BlockDesc));
    L.cols = o;
    o += align256(2 * T * sizeof(MergeDesc));
    L.mom = o;
    o += align256(K * (T + 1) * 9 * sizeof(double));
    L.cvar = o;
    o += align256(K * (T + 1) * (size_t)p.n_con * sizeof(double));
    L.S = o;
    o += align256(K * sizeof(double));
    L.partial = o;
    o += align256((size_t)nblocks * partial_stride(T) * sizeof(double));
    L.total = o;
    return L;
}

}  // namespace

}  // namespace bss

using namespace bss;

extern "C" size_t bss_noalloc_scratch_bytes(const bss_params* p)
{
    if (!p || bss_validate(p) != BSS_OK) return 0;
    const LaunchShape sh = choose_shape(p->K, p->M, p->T, p->lanes, 0, -1, shape_for_shield(*p));
    return layout_of(*p, solve_blocks(p->K, sh.lanes)).total;
}

extern "C" bss_status bss_solve_noalloc(const bss_params* p, uint32_t solve_index,
                                        const double* x0_dev, const double* Sigma0_dev,
                                        const double* v_in_dev, double* v_out_dev,
                                        double* stats_dev, void* stream)
{
    bss_status st = bss_validate(p);
    if (st != BSS_OK) return st;
    if (p->local_repair != 0)
        return fail(BSS_E_INVAL, "bss_solve_noalloc: local_repair is not supported");
    if (!x0_dev || !v_in_dev || !v_out_dev || !stats_dev)
        return fail(BSS_E_INVAL, "bss_solve_noalloc: x0, v_in, v_out and stats must not be NULL");
    if (v_in_dev == v_out_dev)
        return fail(BSS_E_INVAL, "bss_solve_noalloc: v_in and v_out must be distinct buffers");
    if (p->vehicle == 1 && Sigma0_dev)
        return fail(BSS_E_INVAL, "bss_solve_noalloc: vehicle 1 takes a known estimate");
    const LaunchShape sh = choose_shape(p->K, p->M, p->T, p->lanes, 0, -1, shape_for_shield(*p));
    const int nblocks = solve_blocks(p->K, sh.lanes);
    const ScratchLayout L = layout_of(*p, nblocks);
    if (L.total > kNoAllocScratchBytes)
        return fail(BSS_E_INVAL,
                    "bss_solve_noalloc: K=%d, M=%d, T=%d, n_con=%d needs %zu bytes of scratch, "
                    "more than the %zu of the library's static array",
                    p->K, p->M, p->T, p->n_con, L.total, kNoAllocScratchBytes);
    void* base = nullptr;
    hipError_t e = scratch_on_current_device(&base);
    if (e != hipSuccess) return device_fail(e, "bss_solve_noalloc: scratch address");
    char* b = (char*)base;

    InstanceDesc d = make_desc(*p);
    d.lanes = sh.lanes;
    d.ppl = sh.ppl;
    d.nblocks = nblocks;
    if (!samples_shielded(*p)) d.sc.shield_iters = 0;
    d.x0_index = 0;
    d.cur = 0;
    d.vshift = 0;
    d.solve_index = solve_index;
    d.done = 0;
    d.shift_after = 0;
    d.status = 0;
    d.v[0] = const_cast<double*>(v_in_dev);   // read by the solve kernel only
    d.v[1] = v_out_dev;                       // the merge writes v+ here
    d.u = nullptr;
    d.mom = (double*)(b + L.mom);
    d.cvar = p->n_con > 0 ? (double*)(b + L.cvar) : nullptr;
    d.S = (double*)(b + L.S);
    d.partial = (double*)(b + L.partial);
    d.stats = stats_dev;
    InstanceDesc* d_desc = (InstanceDesc*)(b + L.desc);
    BlockDesc* d_blocks = (BlockDesc*)(b + L.blocks);
    MergeDesc* d_cols = (MergeDesc*)(b + L.cols);

    const hipStream_t s = (hipStream_t)stream;
    const bool split = sh.split && !launch_shield(*p) && !launch_resample(*p) &&
                       p->vehicle == 0 &&
                       split_fits(sh.lanes, p->T, sh.ppl, false, p->n_con > 0, kStaticLdsSlots);
    const size_t lds = p->vehicle == 1 ? solve8_lds_bytes(sh.lanes, p->T)
                                       : solve_lds_bytes(sh.lanes, p->T, sh.ppl, split,
                                                         launch_resample(*p), p->n_con > 0);
    hipLaunchKernelGGL(setup_kernel, dim3(1), dim3(256), 0, s, d, d_desc, d_blocks, nblocks,
                       256 / sh.lanes, d_cols, 2 * p->T);
    e = hipGetLastError();
    if (e != hipSuccess) return device_fail(e, "bss_solve_noalloc: set-up launch");
    e = p->vehicle == 1
            ? launch_solve8(d_desc, d_blocks, nblocks, sh.ppl, lds, x0_dev, 0, s)
            : launch_solve(d_desc, d_blocks, nblocks, sh.ppl, launch_shield(*p), split,
                           launch_resample(*p), p->n_con > 0, lds, x0_dev, Sigma0_dev, 0, s);
    if (e != hipSuccess) return device_fail(e, "bss_solve_noalloc: solve launch");
    e = launch_merge(d_desc, d_cols, 2 * p->T, 0, s);
    if (e != hipSuccess) return device_fail(e, "bss_solve_noalloc: merge launch");
    return BSS_OK;
}
