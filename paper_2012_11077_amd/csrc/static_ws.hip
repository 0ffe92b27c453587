// The allocation-free entry point: cfar2d_static runs one map in the TILED
// form (eqs. 1-4, the same kernels as cfar2d) with its workspace -- the work
// counter and the threshold table of eq. (2) -- in a static device array
// instead of caller memory, for callers that cannot allocate.
#include "internal.h"

#include <mutex>

namespace cfar {
namespace {

// Bytes of the static workspace of each device: a 256-byte header (work
// counters, zeroed by the table kernel at every call) and the threshold
// table of up to (kStaticWsBytes - 256) / 8 entries.
constexpr size_t kStaticWsBytes = 1 << 20;

// Every GPU the library runs on holds its own copy until the process ends.
// Host code never uses this name as an address: it takes each device's
// address from hipGetSymbolAddress.
static __device__ __align__(256) char scratch[kStaticWsBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
int scratch_ptr(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return set_error(CFAR_EDEVICE, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return CFAR_OK;
}

}  // namespace
}  // namespace cfar

using namespace cfar;

extern "C" size_t cfar2d_static_max_bytes(void) { return kStaticWsBytes; }

extern "C" int cfar2d_static(const cfar_map *m, void *stream)
{
    int rc = validate_map(m, 0, CFAR_FORM_TILED);
    if (rc != CFAR_OK) return rc;
    const size_t need = tiled_single_ws_bytes(m);
    if (need > kStaticWsBytes)
        return set_error(CFAR_ENOSPC, "window needs %zu workspace bytes, the static workspace holds %zu (at most %zu "
                         "training cells)", need, kStaticWsBytes, (kStaticWsBytes - 256) / 8 - 1);
    void *ws = nullptr;
    rc = scratch_ptr(&ws);
    if (rc != CFAR_OK) return rc;
    return tiled_single_ws(m, ws, kStaticWsBytes, (hipStream_t)stream);
}
