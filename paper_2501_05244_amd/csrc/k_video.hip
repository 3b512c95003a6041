// 4D light transport (eq. Video_Voxel_Freq_Offset): the coherent field of
// every voxel as a function of time,
//   V(x, t_j) = sum_b e^{+j 2 pi f_b t_j} W_b(x),   t_j = t_first + j t_step,
// from the per-frequency fields W_b (back-propagation times illumination
// phase) that the row pass stores for one slab of planes.  One thread per
// voxel keeps kVideoFrames frame accumulators in registers; the block's
// table e^{+j 2 pi f_b t_j} (FP64 argument reduced to a fraction of a cycle)
// sits in LDS and is read as a broadcast.
#include "fft.hpp"
#include "kernels.hpp"

namespace nursd {

constexpr int kVideoThreads = 256;
constexpr int kVideoFrames = 16;     // frames per pass

__global__ __launch_bounds__(kVideoThreads) void k_video(VideoArgs a) {
    extern __shared__ float2 tab[];  // [F][kVideoFrames]
    const int j0 = blockIdx.y * kVideoFrames;
    const int nj = min(kVideoFrames, a.T - j0);
    for (int i = threadIdx.x; i < a.F * kVideoFrames; i += kVideoThreads) {
        const int b = i / kVideoFrames, j = i % kVideoFrames;
        const double cyc = a.f[b] * (a.t_first + (double)(j0 + j) * a.t_step);
        float s, c;
        sincos_cycles((float)(cyc - rint(cyc)), &s, &c);
        tab[i] = make_float2(c, s);
    }
    __syncthreads();
    const int v = blockIdx.x * kVideoThreads + threadIdx.x;
    const int nv = a.nzc * a.nvp;
    if (v >= nv) return;
    const size_t fstride = (size_t)a.field_nz * a.nvp;
    float2 acc[kVideoFrames];
#pragma unroll
    for (int j = 0; j < kVideoFrames; ++j) acc[j] = make_float2(0.f, 0.f);
    float2 w = a.field[v];
    for (int b = 0; b < a.F; ++b) {
        const float2 cur = w;
        if (b + 1 < a.F) w = a.field[(size_t)(b + 1) * fstride + v];
#pragma unroll
        for (int j = 0; j < kVideoFrames; ++j) {
            const float2 e = tab[b * kVideoFrames + j];
            acc[j].x = fmaf(cur.x, e.x, fmaf(-cur.y, e.y, acc[j].x));
            acc[j].y = fmaf(cur.x, e.y, fmaf(cur.y, e.x, acc[j].y));
        }
    }
    const size_t o = (size_t)a.z0 * a.nvp + v;       // plane z0 + v / nvp, pixel v % nvp
    const size_t tstride = (size_t)a.nz * a.nvp;
#pragma unroll
    for (int j = 0; j < kVideoFrames; ++j) {
        const size_t q = (size_t)(j0 + j) * tstride + o;
        if (j < nj && a.V) a.V[q] = acc[j];
        if (j < nj && a.I) a.I[q] = sqrtf(acc[j].x * acc[j].x + acc[j].y * acc[j].y);
    }
}

hipError_t launch_video(const VideoArgs& a, hipStream_t s) {
    if (a.T < 1 || a.nzc < 1) return hipSuccess;
    const dim3 grid((a.nzc * a.nvp + kVideoThreads - 1) / kVideoThreads, (a.T + kVideoFrames - 1) / kVideoFrames);
    const size_t sh = (size_t)a.F * kVideoFrames * sizeof(float2);
    if (sh > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_video, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_video, grid, dim3(kVideoThreads), sh, s, a);
    return hipGetLastError();
}

}  // namespace nursd
