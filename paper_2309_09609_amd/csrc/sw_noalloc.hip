// Allocation-free top-k: the two-launch form of sw_topk_ws with its piece
// workspace in a fixed device array instead of caller or library memory, for
// callers that cannot allocate (graph capture, serving loops).
//
// The array holds the candidates of the first launch (each piece's own top k)
// for the second; it is fully written before it is read, so nothing needs
// clearing between calls.  Every call on a device shares that device's copy of
// the array: calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/swsearch.h"

namespace sw {
hipError_t launch_topk_ws(const int32_t* scores, int64_t n, int64_t row_stride, int rows, int k, int32_t* top_s,
                          int64_t* top_i, void* ws, hipStream_t st);
int64_t topk_ws_bytes(int64_t n, int rows, int k);
sw_status report(sw_status s, const char* fmt, ...);
}  // namespace sw

// 256 pieces x 1024 candidates x (int64 index + int32 score) = 3 MiB + 256 is the most one row needs.
constexpr int64_t kNoAllocBytes = (int64_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void* g_ptr[kMaxDevices];            // the device address of `scratch` on each device
hipError_t g_set[kMaxDevices];

// With device dev current: its copy of the array, looked up once.
hipError_t scratch_on(int dev, void** out) {
    std::call_once(g_once[dev], [dev] {
        void* p = nullptr;
        g_set[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_ptr[dev] = g_set[dev] == hipSuccess ? p : nullptr;
    });
    *out = g_ptr[dev];
    return g_set[dev];
}
}  // namespace

extern "C" sw_status sw_topk_noalloc(const int32_t* d_scores, int64_t n, int32_t k, int32_t* d_top_scores,
                                     int64_t* d_top_index, sw_stream stream) {
    using sw::report;
    report(SW_OK, "");
    if (n < 0) return report(SW_E_INVALID, "n must be >= 0");
    if (k < 1 || k > 1024) return report(SW_E_UNSUPPORTED, "k must be in 1..1024 (got %d)", k);
    if ((n > 0 && !d_scores) || !d_top_scores || !d_top_index) return report(SW_E_INVALID, "NULL pointer");
    const int64_t need = sw::topk_ws_bytes(n, 1, k);
    if (need > kNoAllocBytes)
        return report(SW_E_SIZE, "top-k workspace of %lld bytes exceeds the fixed %lld", (long long)need,
                      (long long)kNoAllocBytes);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return report(SW_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return report(SW_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    void* ws = nullptr;
    if (need > 0) {
        e = scratch_on(dev, &ws);
        if (e != hipSuccess) return report(SW_E_HIP, "hipGetSymbolAddress: %s", hipGetErrorString(e));
    }
    e = sw::launch_topk_ws(d_scores, n, n, 1, k, d_top_scores, d_top_index, need > 0 ? ws : nullptr,
                           static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return report(SW_E_HIP, "top-k launch: %s", hipGetErrorString(e));
    return SW_OK;
}
