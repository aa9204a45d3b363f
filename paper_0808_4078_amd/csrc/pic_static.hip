// pic_init_static_scratch: a run whose scratch is an array the library holds
// on each device, for callers that cannot allocate device memory.
//
// The array is a file-scope __device__ variable, so every device the library
// runs on holds its own copy (until the process ends).  In host code its name
// is only a stand-in: the device address is resolved once per device with
// hipGetSymbolAddress, with that device current, and only that address is
// handed to the kernels (through the run's parameter block, which itself
// lives in the scratch).  A run claims its device's array from
// initialisation to pic_destroy; a second claim is refused, since two runs on
// one array would overwrite each other's state.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pic_internal.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[PIC_STATIC_SCRATCH_BYTES];

std::mutex g_mu;
void *g_ptr[pic::kMaxDevices] = {};   // device address of `scratch` on each device

}  // namespace

extern "C" int pic_init_static_scratch(const pic_grid_desc *grid, const pic_species_desc *species, int nspecies,
                                       const pic_buffers *buffers, void *hip_stream, pic_run **out)
{
    if (!grid || !buffers || !out) return pic::fail_global(PIC_E_INVALID_ARG, "null argument");
    *out = nullptr;
    if (buffers->scratch)
        return pic::fail_global(PIC_E_INVALID_ARG, "buffers->scratch must be NULL: the run uses the library's scratch");
    pic_sizes sz;
    int rc = pic_query(grid, species, nspecies, &sz);
    if (rc) return rc;
    if (sz.scratch_bytes > PIC_STATIC_SCRATCH_BYTES)
        return pic::fail_global(PIC_E_BUFFER_TOO_SMALL, "the run needs %zu bytes of scratch; the library holds %zu",
                                sz.scratch_bytes, (size_t)PIC_STATIC_SCRATCH_BYTES);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return pic::fail_global(PIC_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= pic::kMaxDevices)
        return pic::fail_global(PIC_E_UNSUPPORTED, "device index %d >= %d", dev, pic::kMaxDevices);
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_ptr[dev]) {
            e = hipGetSymbolAddress(&g_ptr[dev], HIP_SYMBOL(scratch));
            if (e != hipSuccess || !g_ptr[dev]) {
                g_ptr[dev] = nullptr;
                return pic::fail_global(PIC_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            }
        }
        ptr = g_ptr[dev];
    }
    if (!pic::claim_static_scratch(dev))
        return pic::fail_global(PIC_E_STATE, "device %d: the library's scratch is held by another run", dev);
    pic_buffers b = *buffers;
    b.scratch = ptr;
    pic_grid_desc g = *grid;
    g.flags |= PIC_FLAG_NO_GRAPH;
    rc = pic::init_run(&g, species, nspecies, &b, hip_stream, out, dev);
    if (rc) pic::release_static_scratch(dev);
    return rc;
}
