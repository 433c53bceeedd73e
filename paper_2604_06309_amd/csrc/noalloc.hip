// dmfe_rhs_noalloc: one right-hand-side evaluation (as dmfe_rhs) whose transient
// buffers live in a static device array instead of the handle's workspace, for
// callers that must not allocate (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation).
//
// The array `scratch` holds, at 256-byte aligned offsets for a grid of L points:
//   the interleaved stage slice y            L YPoint (16 L bytes)
//   the right-hand side before de-interleave L YPoint (16 L bytes)
//   the stage slice in history format        L HPoint (32 L bytes; HPoint32 uses half)
//   its log mirror (log-R option)            L LogPoint (16 L bytes)
//   mu(t), E(t) and the two diagonal values  4 doubles
// so every call fits in 80 L + 4 * 256 bytes; L is limited to kNoallocMaxL.
//
// Host code never uses the array's name as an address: each device's copy is
// found once with hipGetSymbolAddress (with that device current) and the
// pointer kept per device.  Every call on a device shares that device's copy,
// so calls that overlap in time on one device race; the caller serialises them.
#include <mutex>

#include "handle.h"

namespace dmfe {
namespace {

constexpr int kNoallocMaxL = 16384;
constexpr size_t kAlignScratch = 256;
constexpr size_t align_s(size_t x) { return (x + kAlignScratch - 1) / kAlignScratch * kAlignScratch; }
constexpr size_t kScratchBytes = align_s(sizeof(YPoint) * kNoallocMaxL) * 2 + align_s(sizeof(HPoint) * kNoallocMaxL) +
                                 align_s(sizeof(LogPoint) * kNoallocMaxL) + kAlignScratch;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// Address of this device's copy of `scratch` (the device must be current).
dmfe_status device_scratch(int dev, char** out) {
    if (dev < 0 || dev >= kMaxDevices) return core::fail_msg(DMFE_ERR_INVALID, "noalloc: device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return core::fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return core::fail_msg(DMFE_ERR_DEVICE, "noalloc: null scratch address");
        g_scratch[dev] = static_cast<char*>(p);
    }
    *out = g_scratch[dev];
    return DMFE_OK;
}

}  // namespace
}  // namespace dmfe

using namespace dmfe;
using namespace dmfe::core;

extern "C" {

dmfe_status dmfe_rhs_noalloc(dmfe_handle* h, double t, const double* yC, const double* yR, int64_t nb,
                             double* outC, double* outR, double* mu, double* diag) {
    if (!h || h->p.mode != DMFE_ADAPTIVE || !yC || !yR || !outC || !outR) return DMFE_ERR_INVALID;
    if (nb < 0 || nb > h->M) return DMFE_ERR_INVALID;
    if (nb > 0 && !(t >= h->thist[nb - 1])) return DMFE_ERR_INVALID;
    if (nb == 0 && t != 0.0) return DMFE_ERR_INVALID;
    const int L = h->L;
    if (L > kNoallocMaxL) return fail_msg(DMFE_ERR_INVALID, "dmfe_rhs_noalloc: L above the scratch limit 16384");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return fail(e, "hipSetDevice");
    char* base = nullptr;
    const dmfe_status ss = device_scratch(h->device, &base);
    if (ss != DMFE_OK) return ss;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base + off;
        off += align_s(bytes);
        return p;
    };
    YPoint* y = reinterpret_cast<YPoint*>(take(sizeof(YPoint) * L));
    YPoint* k = reinterpret_cast<YPoint*>(take(sizeof(YPoint) * L));
    StageBufs b{};
    b.stage = take(point_bytes(h) * L);
    LogPoint* lst = reinterpret_cast<LogPoint*>(take(sizeof(LogPoint) * L));
    b.lstage = h->p.log_r ? lst : nullptr;
    double* small = reinterpret_cast<double*>(take(4 * sizeof(double)));
    b.mue = small;
    b.diag = small + 2;
    HCHK(launch_interleave(L, yC, yR, y, h->stream));
    const dmfe_status st = eval_rhs(h, t, int(nb), y, k, nullptr, b, false);
    if (st != DMFE_OK) return st;
    HCHK(launch_deinterleave(L, k, outC, outR, h->stream));
    HCHK(hipMemcpyAsync(h->pinned, small, 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HCHK(hipStreamSynchronize(h->stream));
    if (mu) *mu = h->pinned[0];
    if (diag) {
        diag[0] = h->pinned[2];
        diag[1] = h->pinned[3];
    }
    return DMFE_OK;
}

}  // extern "C"
