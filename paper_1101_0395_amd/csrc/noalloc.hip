// cq_quantize_noalloc: the whole quantizer of one image without any memory
// allocation, for callers that cannot allocate (code under graph capture,
// tight serving loops, harnesses that forbid it).  Its workspace is a fixed
// array in device memory, `scratch`, of kScratchBytes, which holds the
// workspace of any image of at most kScratchPixels pixels; each GPU the
// library runs on holds its own copy until the process ends.  Host-side
// staging goes through a fixed pageable array, and the events of the
// status readback are created once per device, on the first call there.
#include <string.h>

#include <map>
#include <mutex>

#include "batch.h"

namespace cq {

constexpr int64_t kScratchPixels = int64_t(1) << 20;          // 1024 x 1024
constexpr size_t kScratchBytes = size_t(48) << 20;             // 48 MiB
constexpr size_t kHostStageBytes = 64 << 10;                   // descriptors and status records of one job

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
struct DeviceSetup {
    void* scratch = nullptr;  // this device's copy of `scratch`
    hipEvent_t ev[2] = {nullptr, nullptr};
};
std::mutex g_setup_mu;
std::map<int, DeviceSetup> g_setup;
// Host staging of the calls; calls from several host threads are serialized
// on g_call_mu (they would race on one GPU's scratch anyway).
std::mutex g_call_mu;
alignas(256) char g_host_stage[kHostStageBytes];
}  // namespace

// The current device's scratch address and readback events, set up on the
// first call on that device (the name `scratch` is a host-side stand-in; the
// device address comes from hipGetSymbolAddress).
static cq_status device_setup(DeviceSetup** out)
{
    int dev = 0;
    CQ_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_setup_mu);
    auto it = g_setup.find(dev);
    if (it == g_setup.end()) {
        DeviceSetup d;
        CQ_HIP_TRY(hipGetSymbolAddress(&d.scratch, HIP_SYMBOL(scratch)));
        if ((reinterpret_cast<uintptr_t>(d.scratch) & 255u) != 0) {
            set_error("scratch array is not 256-byte aligned");
            return CQ_EDEVICE;
        }
        for (auto& e : d.ev) CQ_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        hipStream_t side = nullptr;
        CQ_TRY(side_stream(&side));  // created now, not during a later call
        it = g_setup.emplace(dev, d).first;
    }
    *out = &it->second;
    return CQ_OK;
}

void noalloc_release()
{
    std::lock_guard<std::mutex> lock(g_setup_mu);
    for (auto& kv : g_setup)
        for (auto e : kv.second.ev)
            if (e) (void)hipEventDestroy(e);
    g_setup.clear();
}

}  // namespace cq

using namespace cq;

extern "C" {

cq_status cq_quantize_noalloc(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride_bytes, int32_t subsample,
                              int32_t K, cq_init_t scheme, uint64_t seed, int32_t max_iters, double tol,
                              int32_t prune, uint8_t* palette, uint8_t* out_idx, uint8_t* out_rgb,
                              cq_stats* stats, void* stream)
{
    clear_error();
    if (H > 0 && W > 0 && int64_t(H) * W > kScratchPixels)
        return einval("image has %lld pixels, more than the %lld that cq_quantize_noalloc's fixed scratch holds",
                      (long long)(int64_t(H) * W), (long long)kScratchPixels);
    const size_t need = cq_workspace_bytes(H, W, K);
    if (need > kScratchBytes) {
        set_error("image needs %zu workspace bytes, the fixed scratch has %zu", need, kScratchBytes);
        return CQ_EWORKSPACE;
    }
    DeviceSetup* d = nullptr;
    CQ_TRY(device_setup(&d));
    std::lock_guard<std::mutex> lock(g_call_mu);
    return quantize_into(img, H, W, row_stride_bytes, subsample, K, scheme, seed, max_iters, tol, prune, palette,
                         out_idx, out_rgb, stats, d->scratch, kScratchBytes, stream, g_host_stage,
                         kHostStageBytes, d->ev);
}

}  // extern "C"
