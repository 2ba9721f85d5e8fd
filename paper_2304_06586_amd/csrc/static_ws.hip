// Allocation-free single solve: gfdtd_solve with its workspace in a fixed
// device array that the library holds on every GPU it runs on, for callers
// that cannot allocate device memory.
//
// The array is a file-scope __device__ variable.  In host code its name is
// only a host-side stand-in, so its device address is looked up once per
// device with hipGetSymbolAddress (with that device current) and that
// address is what the batch carves and the kernels receive.  Calls are
// serialised per device inside the process: every call on a GPU reuses
// that GPU's array, and it keeps the last call's contents (every pass
// re-zeroes the fields and rewrites every other array it reads before
// reading it).
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>

#include "gfdtd.h"
#include "gfdtd_internal.h"
#include "runtime.h"

namespace gfdtd {

namespace {

constexpr size_t kScratchBytes = GFDTD_STATIC_WORKSPACE_BYTES;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
    void *ptr = nullptr;      // device address of `scratch` on this device
    std::mutex run;           // one solve at a time per device
};

std::mutex g_table_mutex;
std::map<int, std::unique_ptr<DeviceScratch>> g_table;

// The device's copy of the array (looked up on its first use), or null
// with the error recorded.
DeviceScratch *device_scratch(int dev)
{
    std::lock_guard<std::mutex> lk(g_table_mutex);
    auto it = g_table.find(dev);
    if (it != g_table.end())
        return it->second.get();
    std::unique_ptr<DeviceScratch> d(new DeviceScratch);
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                 "look up the static workspace");
        return nullptr;
    }
    d->ptr = p;
    DeviceScratch *raw = d.get();
    g_table[dev] = std::move(d);
    return raw;
}

}  // namespace

}  // namespace gfdtd

using namespace gfdtd;

extern "C" {

gfdtd_status gfdtd_solve_static(const gfdtd_problem *p, int64_t steps, void *stream,
                                gfdtd_result *out)
{
    clear_error();
    if (!p || !out)
        return fail(GFDTD_E_INVALID, "problem or result is NULL");
    if (out->struct_size < sizeof(gfdtd_result))
        return fail(GFDTD_E_INVALID, "result struct_size too small");
    // size check first: an oversized problem is rejected before any device call
    size_t need = 0;
    gfdtd_status st = gfdtd_workspace_bytes(p, steps, &need);
    if (st != GFDTD_OK)
        return st;
    if (need > kScratchBytes)
        return fail(GFDTD_E_NOMEM,
                    "problem needs a %zu-byte workspace; the static workspace holds "
                    "%zu bytes (use gfdtd_solve with a caller workspace)",
                    need, kScratchBytes);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "current device");
    DeviceScratch *ds = device_scratch(dev);
    if (!ds)
        return GFDTD_E_DEVICE;
    std::lock_guard<std::mutex> lk(ds->run);
    gfdtd_exec ex{};
    ex.struct_size = sizeof(gfdtd_exec);
    ex.variant = GFDTD_VARIANT_AUTO;
    ex.use_graph = 0;                  // no graph: capture would allocate
    Batch b;
    b.no_alloc = true;
    st = b.prepare(p, &steps, 1, &ex, ds->ptr, kScratchBytes,
                   static_cast<hipStream_t>(stream));
    if (st == GFDTD_OK)
        st = b.run();
    if (st == GFDTD_OK)
        st = b.collect(out);
    return st;
}

}  // extern "C"
