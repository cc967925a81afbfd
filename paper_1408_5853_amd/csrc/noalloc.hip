// cryo_forward_noalloc: the forward of cryo_forward with its workspace in a
// library-owned device array instead of caller memory, for callers that
// cannot allocate (code under HIP graph capture, tight serving loops).
//
// The array lives in this code object's device data: each GPU the library
// runs on holds its own copy, at its own address, until the process ends.
// In host code the array's name is only a host-side stand-in, so its device
// address is looked up once per device (hipGetSymbolAddress, with that device
// current) and only that address is handed to kernels.
#include <mutex>

#include "internal.h"

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)CRYO_NOALLOC_MAX_BYTES;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on device `dev` (current), looked up on the
// first use on that device.
cryo_status scratch_on(int dev, char **out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return cryo::fail(CRYO_ERR_DEVICE,
                              std::string("scratch address: ") + hipGetErrorString(e));
        g_ptr[dev] = ptr;
    }
    *out = (char *)g_ptr[dev];
    return CRYO_OK;
}

}  // namespace

extern "C" {

cryo_status cryo_forward_noalloc(const cryo_plan *p, void *T, int64_t k0, int64_t nsteps,
                                 double *surf, void *stream) {
    using cryo::fail;
    if (!p || !T || nsteps < 0 || k0 < 0) return fail(CRYO_ERR_ARG, "bad argument");
    size_t need = 0;
    cryo_status st = cryo_workspace_bytes(p, 0, &need);
    if (st != CRYO_OK) return st;
    if (need > SCRATCH_BYTES)
        return fail(CRYO_ERR_WORKSPACE,
                    "cryo_forward_noalloc: the cell needs " + std::to_string(need) +
                        " bytes of workspace, above the built-in scratch of " +
                        std::to_string(SCRATCH_BYTES) + " bytes (use cryo_forward)");
    if (!cryo::plan_tables_on_device(p))
        return fail(CRYO_ERR_ARG, "cryo_forward_noalloc: the plan has no device tables yet "
                                  "(make them once with cryo_state_create or cryo_forward)");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
        return fail(CRYO_ERR_DEVICE, "cryo_forward_noalloc: no current device");
    if (dev != p->device)
        return fail(CRYO_ERR_ARG, "cryo_forward_noalloc: the current device is not the "
                                  "plan's device");
    char *w = nullptr;
    st = scratch_on(dev, &w);
    if (st != CRYO_OK) return st;
    return cryo::forward_in(p, T, k0, nsteps, w, surf, (hipStream_t)stream);
}

}  // extern "C"
