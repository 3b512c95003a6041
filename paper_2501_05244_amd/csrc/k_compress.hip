// Compression preprocessing of the sampling-criteria section: the relay-grid
// phasors are kept on the lattice of stride D per axis (the rest discarded)
// and every grid point is filled from its nearest kept sample.  On a product
// lattice the nearest point is found axis by axis: i -> D * round(i / D) with
// halves rounded down (ties go to the lower kept index), clamped to the last
// kept index.  Pure index arithmetic: the output is a bit-exact gather.
#include "kernels.hpp"

namespace nursd {

__device__ __forceinline__ int nearest_kept(int i, int n, int D) {
    const int q = (2 * i + D - 1) / (2 * D) * D;
    const int last = (n - 1) / D * D;
    return q < last ? q : last;
}

__global__ __launch_bounds__(256) void k_subsample_nearest(const float2* __restrict__ in, float2* __restrict__ out,
                                                           int F, int ny, int nx, int D) {
    const size_t n = (size_t)F * ny * nx;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const int ix = (int)(i % nx);
        const size_t r = i / nx;
        const int iy = (int)(r % ny);
        const size_t b = r / ny;
        out[i] = in[(b * ny + nearest_kept(iy, ny, D)) * nx + nearest_kept(ix, nx, D)];
    }
}

hipError_t launch_subsample_nearest(const float2* in, float2* out, int F, int ny, int nx, int D, hipStream_t s) {
    const size_t n = (size_t)F * ny * nx;
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_subsample_nearest, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, in,
                       out, F, ny, nx, D);
    return hipGetLastError();
}

}  // namespace nursd
