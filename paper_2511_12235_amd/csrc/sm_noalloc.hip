// sm_noalloc.hip -- sm_apply_noalloc: the operators of sm_forward / sm_back
// for callers that cannot allocate device memory (code under stream capture,
// serving loops, hosts that forbid hipMalloc).  The workspace those entry
// points take from the caller (strip records of a chunk of views, the
// forward's prefix sums, the adjoint's partial volumes) lives here in one
// file-scope device array, `scratch`, of kScratchBytes per device.
//
// The array is a host-side stand-in in host code: its device address is
// looked up once per device with hipGetSymbolAddress (on the first call made
// with that device current) and only that address is handed to kernels.
// Every call on a device uses the same array, so calls that overlap in time on
// one device (several streams or host threads) race; the array keeps the last
// call's contents.  No kernel reads scratch memory it has not written in the
// same call, so nothing is cleared between calls.
#include <mutex>

#include "sm_plan.h"

namespace {
constexpr int64_t kScratchBytes = SM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` on each device, once looked up

// Device address of `scratch` on device `dev`, which must be current.
sm_status scratch_address(int dev, char **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return smk::set_error(SM_EUNSUPPORTED, "device %d: scratch addresses are kept for %d devices",
                              dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return smk::set_error(SM_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                                  hipGetErrorString(e));
        g_scratch[dev] = ptr;
    }
    *out = (char *)g_scratch[dev];
    return SM_OK;
}

}  // namespace

extern "C" {

sm_status sm_apply_noalloc(const sm_plan *p, int32_t adjoint, const void *in, void *out,
                           int32_t batch, void *hip_stream)
{
    sm_status s = smk::check_operands(p, in, out, batch);
    if (s != SM_OK) return s;
    if (adjoint != 0 && adjoint != 1) return smk::set_error(SM_EINVAL, "adjoint must be 0 or 1");
    hipStream_t st = (hipStream_t)hip_stream;
    const char *what = adjoint ? "sm_apply_noalloc (adjoint)" : "sm_apply_noalloc (forward)";
    if (p->G.dim == 2) {  // the 2D operators need no workspace
        const hipError_t e = smk::run_apply2d(p, adjoint != 0, in, out, batch, st);
        return e == hipSuccess ? SM_OK : smk::set_error(SM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    }
    // Volume buffer first: the adjoint drops view runs (partial volumes, the
    // rounding order of its sums) until one chunk of a view's records fits
    // beside them; then as many views per chunk as fit.
    smk::LaunchCfg L = p->L;
    const size_t rsz = p->prec == SM_FP64 ? sizeof(smk::Rec<double>) : sizeof(smk::Rec<float>);
    auto layout = [&](int views) {
        return smk::make_layout(p->RL.cap, p->RL.n_major_max, views, p->G.nu, p->G.nx, p->G.ny, rsz);
    };
    const int64_t one_view = p->rec_cache ? 0 : layout(1).data_off;
    int64_t vol = adjoint ? smk::back_volume_bytes(p, batch, L.back_groups) : smk::fwd_volume_bytes(p, batch);
    while (adjoint && L.back_groups > 1 && one_view + vol > kScratchBytes) {
        --L.back_groups;
        vol = smk::back_volume_bytes(p, batch, L.back_groups);
    }
    if (one_view + vol > kScratchBytes)
        return smk::set_error(SM_ERANGE,
                              "%s needs %lld bytes of scratch (%lld of volume buffers, %lld of strip "
                              "records of one view), more than the %lld bytes of the static scratch "
                              "array; use %s with a workspace", what, (long long)(one_view + vol),
                              (long long)vol, (long long)one_view, (long long)kScratchBytes,
                              adjoint ? "sm_back" : "sm_forward");
    smk::RecLayout RL = p->RL;  // kept records: the plan's chunks
    if (!p->rec_cache) {
        int lo = 1, hi = p->RL.views;  // largest view count that fits
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (layout(mid).data_off + vol <= kScratchBytes) lo = mid; else hi = mid - 1;
        }
        // equal chunks, as the plan's own layout
        const int chunks = (p->G.n_p + lo - 1) / lo;
        RL = layout((p->G.n_p + chunks - 1) / chunks);
    }
    char *base = nullptr;
    s = scratch_address(p->device, &base);
    if (s != SM_OK) return s;
    char *volp = base + (p->rec_cache ? 0 : RL.data_off);
    const hipError_t e = adjoint ? smk::run_back3d(p, RL, L, in, out, batch, base, volp, st)
                                 : smk::run_forward3d(p, RL, in, out, batch, base, volp, st);
    return e == hipSuccess ? SM_OK : smk::set_error(SM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // extern "C"
