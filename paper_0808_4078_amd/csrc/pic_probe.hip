// Bandwidth probe of libpic (measurement only, no part of a step): a copy of
// several arrays of 4-byte words in one launch, lane i copying word i of each
// array in turn -- the access pattern of the particle kernel's state streams
// (one SoA stream per quantity, 4-byte lanes) without its arithmetic, binning
// or LDS work.  Its rate is the practical copy ceiling of that pattern.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace pic {

struct CopyArrays {
    const uint32_t *src[8];
    uint32_t *dst[8];
};

template <int NA>
__global__ __launch_bounds__(256) void k_copy_probe(CopyArrays a, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t v[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) v[k] = a.src[k][i];
#pragma unroll
        for (int k = 0; k < NA; ++k) a.dst[k][i] = v[k];
    }
}

// narrays in 1..8 and n >= 1 (checked by the caller); 64 workgroups of 256
// per compute unit at most, each lane striding over the arrays
hipError_t launch_copy_probe(const uint32_t *const *src, uint32_t *const *dst, int narrays, int64_t n,
                             hipStream_t st)
{
    CopyArrays a{};
    for (int k = 0; k < narrays; ++k) {
        a.src[k] = src[k];
        a.dst[k] = dst[k];
    }
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 256 * 64);
    switch (narrays) {
    case 1: hipLaunchKernelGGL(k_copy_probe<1>, dim3(blocks), dim3(256), 0, st, a, n); break;
    case 2: hipLaunchKernelGGL(k_copy_probe<2>, dim3(blocks), dim3(256), 0, st, a, n); break;
    case 3: hipLaunchKernelGGL(k_copy_probe<3>, dim3(blocks), dim3(256), 0, st, a, n); break;
    case 4: hipLaunchKernelGGL(k_copy_probe<4>, dim3(blocks), dim3(256), 0, st, a, n); break;
    case 5: hipLaunchKernelGGL(k_copy_probe<5>, dim3(blocks), dim3(256), 0, st, a, n); break;
    case 6: hipLaunchKernelGGL(k_copy_probe<6>, dim3(blocks), dim3(256), 0, st, a, n); break;
    case 7: hipLaunchKernelGGL(k_copy_probe<7>, dim3(blocks), dim3(256), 0, st, a, n); break;
    case 8: hipLaunchKernelGGL(k_copy_probe<8>, dim3(blocks), dim3(256), 0, st, a, n); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace pic
