// Bandwidth probe of libpic (measurement only, no part of a step): a copy of
// several arrays of 4-byte words in one launch, each workgroup streaming one
// chunk of every array -- the access pattern of the particle kernel's state
// streams (one SoA stream per quantity, 4-byte lanes, a workgroup per tile's
// bin) without its arithmetic, binning or LDS work.  Its rate is the
// practical copy ceiling of that pattern at a given chunk length.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace pic {

struct CopyArrays {
    const uint32_t *src[8];
    uint32_t *dst[8];
};

template <int NA>
__global__ __launch_bounds__(256) void k_copy_probe(CopyArrays a, int64_t n, int64_t chunk)
{
    // workgroup b copies words [b chunk, (b + 1) chunk) of every array, 256 at a time
    const int64_t b0 = (int64_t)blockIdx.x * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) {
        uint32_t v[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) v[k] = a.src[k][i];
#pragma unroll
        for (int k = 0; k < NA; ++k) a.dst[k][i] = v[k];
    }
}

// narrays in 1..8, n >= 1, chunk a positive multiple of 256 (checked by the
// caller); one workgroup of 256 per chunk of each array
hipError_t launch_copy_probe(const uint32_t *const *src, uint32_t *const *dst, int narrays, int64_t n,
                             int64_t chunk, hipStream_t st)
{
    CopyArrays a{};
    for (int k = 0; k < narrays; ++k) {
        a.src[k] = src[k];
        a.dst[k] = dst[k];
    }
    const int64_t nb = (n + chunk - 1) / chunk;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)nb;
    switch (narrays) {
    case 1: hipLaunchKernelGGL(k_copy_probe<1>, dim3(blocks), dim3(256), 0, st, a, n, chunk); break;
    case 2: hipLaunchKernelGGL(k_copy_probe<2>, dim3(blocks), dim3(256), 0, st, a, n, chunk); break;
    case 3: hipLaunchKernelGGL(k_copy_probe<3>, dim3(blocks), dim3(256), 0, st, a, n, chunk); break;
    case 4: hipLaunchKernelGGL(k_copy_probe<4>, dim3(blocks), dim3(256), 0, st, a, n, chunk); break;
    case 5: hipLaunchKernelGGL(k_copy_probe<5>, dim3(blocks), dim3(256), 0, st, a, n, chunk); break;
    case 6: hipLaunchKernelGGL(k_copy_probe<6>, dim3(blocks), dim3(256), 0, st, a, n, chunk); break;
    case 7: hipLaunchKernelGGL(k_copy_probe<7>, dim3(blocks), dim3(256), 0, st, a, n, chunk); break;
    case 8: hipLaunchKernelGGL(k_copy_probe<8>, dim3(blocks), dim3(256), 0, st, a, n, chunk); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace pic
