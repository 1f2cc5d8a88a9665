// grid_check.hip -- device-side check of the tensor-grid statement of an occupancy.
//
// An occupancy whose `grid` field is set is evaluated through the per-axis
// factorisation, which reads only the axis entries of the hinge array (X0[i] = h[i],
// X1[i] = h[M + g0 i], X2[i] = h[2M + g0 g1 i]).  Before such a launch the entry
// points enqueue this check on the same stream: every hinge j = i0 + g0 (i1 + g1 i2)
// must equal (X0[i0], X1[i1], X2[i2]) (by value; a NaN coordinate fails).  A mismatch
// sets a sticky per-device word that pdmp_sync reports as PDMP_EINVAL and clears;
// the launch itself runs to completion (its results are then undefined).
#include "pdmp_common.h"

namespace pdmp {

__device__ uint32_t g_grid_mismatch = 0;

__global__ void __launch_bounds__(256)
k_grid_check(const float *__restrict__ h, int dim, int M, int g0, int g1) {
    bool ok = true;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < M; j += gridDim.x * blockDim.x) {
        const int i0 = j % g0, r = j / g0, i1 = r % g1, i2 = r / g1;
        ok = ok && h[j] == h[i0];
        ok = ok && h[(size_t)M + j] == h[(size_t)M + (size_t)g0 * i1];
        if (dim == 3) ok = ok && h[2 * (size_t)M + j] == h[2 * (size_t)M + (size_t)g0 * g1 * i2];
    }
    if (__any(!ok) && (threadIdx.x & 63) == 0) atomicOr(&g_grid_mismatch, 1u);
}

int32_t launch_grid_check(int dim, const float *hinges, int M, const int *grid, hipStream_t st) {
    const int blocks = (M + 255) / 256 < 64 ? (M + 255) / 256 : 64;
    hipLaunchKernelGGL(k_grid_check, dim3(blocks), dim3(256), 0, st, hinges, dim, M, grid[0],
                       grid[1]);
    return check_launch("k_grid_check");
}

// Reads and clears the current device's mismatch word (host-synchronous).
int32_t take_grid_mismatch(bool &mismatch) {
    uint32_t v = 0;
    hipError_t e = hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_grid_mismatch), sizeof(v), 0,
                                       hipMemcpyDeviceToHost);
    if (e == hipSuccess && v != 0) {
        const uint32_t zero = 0;
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_grid_mismatch), &zero, sizeof(zero), 0,
                              hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        set_error("grid check word: %s", hipGetErrorString(e));
        return PDMP_EDEVICE;
    }
    mismatch = v != 0;
    return PDMP_OK;
}

}  // namespace pdmp
