// reconstruct_hybrid for callers that cannot allocate device memory: its
// workspace (scan spectrum, range profiles, image spectrum, plan tables) is
// a file-scope device array of PL_STATIC_SCRATCH_BYTES, one copy per device,
// held until the process ends.  Host code never uses the array's name as an
// address (on the host it is only a stand-in): the device address of the
// current device's copy is looked up once per device and passed to the
// kernels like any workspace.
#include "internal.hpp"

namespace pl {
namespace {

static __device__ __align__(256) unsigned char scratch[PL_STATIC_SCRATCH_BYTES];

// Device address of this device's copy of `scratch`, from
// hipGetSymbolAddress with the device current, cached per device.
int scratch_address(void** out) {
    static std::mutex mu;
    static std::map<int, void*> addr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(PL_EDEVICE, "reconstruct_hybrid_static: hipGetDevice: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) {
        *out = it->second;
        return PL_OK;
    }
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(PL_EDEVICE, "reconstruct_hybrid_static: scratch address on device %d: %s", dev,
                    hipGetErrorString(e));
    if ((reinterpret_cast<uintptr_t>(p) & 255u) != 0)
        return fail(PL_EDEVICE, "reconstruct_hybrid_static: scratch on device %d is not 256-byte aligned", dev);
    addr[dev] = p;
    *out = p;
    return PL_OK;
}

}  // namespace
}  // namespace pl

extern "C" int reconstruct_hybrid_static(const pl_geometry* g, const pl_image_grid* grid, const pl_hybrid_opts* opts,
                                         const float* echo, float* image, hipStream_t stream) {
    using namespace pl;
    clear_error();
    if (!g || !grid || !echo || !image) return fail(PL_EINVAL, "reconstruct_hybrid_static: null argument");
    HybridPlan p;
    int rc = make_plan(g, grid, opts, &p);
    if (rc) return rc;
    if (p.total > static_cast<size_t>(PL_STATIC_SCRATCH_BYTES))
        return fail(PL_EWORKSPACE,
                    "reconstruct_hybrid_static: this problem needs %zu bytes of workspace, the static scratch "
                    "holds %zu (use reconstruct_hybrid with a workspace)",
                    p.total, static_cast<size_t>(PL_STATIC_SCRATCH_BYTES));
    void* ws = nullptr;
    if ((rc = scratch_address(&ws))) return rc;
    return reconstruct_impl(g, grid, opts, echo, image, ws, PL_STATIC_SCRATCH_BYTES, nullptr, stream, true, false,
                            "reconstruct_hybrid_static");
}
