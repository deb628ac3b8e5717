// sre2_noalloc.hip - sre2_m2_noalloc: one M2 evaluation whose intermediate
// buffers live in a fixed, file-scope device array instead of memory the
// library allocates (include/sre2.h).  The launch sequence and kernels are
// those of sre2_m2 (sre2::ws_m2).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/sre2.h"
#include "sre2_ctx.h"

namespace {

constexpr size_t kScratchBytes = SRE2_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The device array.  In host code `scratch` names a host-side stand-in, not
// a device address: only the per-device address from hipGetSymbolAddress is
// ever passed to the kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_addr[kMaxDevices] = {};  // device address of `scratch` on each device

// Device address of `scratch` on `dev`, which must be the current device;
// looked up once per device.
int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return SRE2_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return SRE2_EHIP;
        }
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    return SRE2_OK;
}

}  // namespace

extern "C" int sre2_m2_noalloc(int hip_device, const void* psi, int N, int dtype, int form,
                               void* stream, double* out, double* partials) {
    if (hip_device < 0 || hip_device >= kMaxDevices || !psi || !out) return SRE2_EINVAL;
    int rc = sre2::ctx_validate_form(N, dtype, form);
    if (rc) return rc;
    size_t o_work = 0, o_sx = 0, o_part = 0, o_slab = 0, limit = 0;
    rc = sre2::ws_layout(N, dtype, form, partials == nullptr, kScratchBytes, &o_work, &o_sx,
                         &o_part, &o_slab, &limit);
    if (rc) return rc;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return SRE2_EHIP;
    if (prev != hip_device && hipSetDevice(hip_device) != hipSuccess) return SRE2_EHIP;
    void* base = nullptr;
    rc = scratch_address(hip_device, &base);
    if (!rc) {
        char* b = static_cast<char*>(base);
        sre2::Workspace ws;
        ws.red = reinterpret_cast<double*>(b);
        ws.psi_work = o_work ? b + o_work : nullptr;
        ws.sx = o_sx ? reinterpret_cast<double*>(b + o_sx) : nullptr;
        ws.part = o_part ? reinterpret_cast<double*>(b + o_part) : nullptr;
        ws.scratch = o_slab ? b + o_slab : nullptr;
        ws.limit = limit;
        rc = sre2::ws_m2(ws, psi, N, dtype, form, (hipStream_t)stream, out, partials);
    }
    if (prev != hip_device) (void)hipSetDevice(prev);
    return rc;
}
