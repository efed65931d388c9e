// dmcr_loss_grad_noalloc: dmcr_loss_grad with its scratch memory taken from a
// fixed device array of this library instead of a caller workspace, for callers
// that cannot allocate (code under stream capture, serving loops that must not
// call the allocator).  The array is a file-scope __device__ variable: every
// device the library runs on holds one copy until the process ends.  Host code
// never uses the array's name as an address: its device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and the
// kernels receive that pointer, exactly as they receive a caller's workspace.
#include <mutex>

#include "dmcr_internal.h"

namespace dmcr {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// the device address of the current device's copy of `scratch`
dmcr_status scratch_of_current_device(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return DMCR_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DMCR_EDEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DMCR_OK;
}

}  // namespace
}  // namespace dmcr

using namespace dmcr;

extern "C" dmcr_status dmcr_loss_grad_noalloc(const dmcr_spec *spec, int32_t batch, const float *phi,
                                              const double *S_target, double *E, float *grad, hipStream_t stream)
{
    Plan p;
    dmcr_status s = make_plan(spec, batch, &p);
    if (s != DMCR_OK) return s;
    if (!phi || !S_target || !E || !grad) return DMCR_EINVAL;
    if (!aligned8(phi) || !aligned8(grad) || !aligned8(S_target) || !aligned8(E)) return DMCR_EINVAL;
    if (p.bytes > kScratchBytes) return DMCR_ENOMEM;
    void *ws = nullptr;
    if ((s = scratch_of_current_device(&ws)) != DMCR_OK) return s;
    // one stream, no internal streams or events: nothing is created or allocated
    return loss_grad_internal(p, phi, S_target, E, grad, Ws{static_cast<char *>(ws)}, stream, false);
}
