// The allocation-free probed gradient (tpx_gradient_probed_noalloc): its
// workspace is a static device array of this library, so the call needs no
// device allocation by anyone.  Each GPU holds its own copy of the array for
// the life of the process; host code reaches a device's copy only through the
// address hipGetSymbolAddress returns with that device current.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "tpx.h"
#include "tpx_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)TPX_NOALLOC_SCRATCH_BYTES;

// The workspace of every allocation-free call on a GPU (one copy per device).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;   // per device: the device address of its copy, or null

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current.
tpx_status scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0) {
        tpx::set_error(TPX_E_DEVICE, (std::string("hipGetDevice: ") + hipGetErrorString(e)).c_str());
        return TPX_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            tpx::set_error(TPX_E_DEVICE,
                           (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
            return TPX_E_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TPX_OK;
}

}  // namespace

extern "C" tpx_status tpx_gradient_probed_noalloc(const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe,
                                                  const float *m, const float *d_obs, float *g, double *J,
                                                  float *d_out, void *stream) {
    void *ws = nullptr;
    const tpx_status st = scratch_address(&ws);
    if (st != TPX_OK) return st;
    return tpx::gradient_probed_in_scratch(grid, geom, probe, m, d_obs, g, J, d_out, ws, kScratchBytes, stream);
}
