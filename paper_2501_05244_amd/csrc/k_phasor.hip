// Step 1: temporal phasor transform.
//
// Per relay sample l and kept DFT bin b:
//   P[b][l] = w(f_b) e^{-j 2 pi f_b t0} sum_t H[l][t] e^{-j 2 pi b t / T}
// (the phasor-field response of eq. PF_Response with the Gaussian
// band-pass illumination of eq. PFPacket_Omega_Supp).  The real T-point
// transform is computed as one T/2-point complex FFT of z[t] = h[2t] + j h[2t+1]
// in LDS, then split: X[b] = E[b] + e^{-j 2 pi b/T} O[b] with
// E = (Z[b] + conj Z[T/2-b]) / 2 and O = (Z[b] - conj Z[T/2-b]) / (2j).
// HBM-bound: each histogram is read once, F values written per sample.
#include "fft.hpp"
#include "kernels.hpp"
#include "persistent.hpp"

namespace nursd {

constexpr int kPhasorThreads = 256;
constexpr int kPhasorGroup = 16;   // relay samples per workgroup (coalesced P writes)

template <int TH>
__device__ __forceinline__ void phasor_body(const PhasorArgs& a, int bx) {
    extern __shared__ float2 smem[];
    float2* line = smem;             // [TH]
    float2* out = smem + TH;         // [F][kPhasorGroup]
    const int l0 = bx * kPhasorGroup;
    const int tid = threadIdx.x;
    for (int r = 0; r < kPhasorGroup; ++r) {
        const int l = l0 + r;
        if (l >= a.L) break;                                    // uniform
        const float2* row = reinterpret_cast<const float2*>(a.hist + (size_t)l * a.T);
        for (int t = tid; t < TH; t += kPhasorThreads) line[t] = row[t];
        __syncthreads();
        fft_lines<TH, kPhasorThreads, false>(line, TH, 1, a.tw);
        for (int j = tid; j < a.F; j += kPhasorThreads) {
            const int b = a.bins[j];
            const float2 zb = line[b];
            const float2 zc = cconj(line[TH - b]);
            const float2 e = cscale(cadd(zb, zc), 0.5f);
            const float2 d = cscale(csub(zb, zc), 0.5f);           // = j * O
            const float2 o = make_float2(d.y, -d.x);               // O = d / j
            const float2 x = cadd(e, cmul(a.tb[j], o));
            out[j * kPhasorGroup + r] = cmul(a.wt[j], x);
        }
        __syncthreads();
    }
    const int nr = min(kPhasorGroup, a.L - l0);
    for (int i = tid; i < a.F * kPhasorGroup; i += kPhasorThreads) {
        const int j = i / kPhasorGroup, r = i % kPhasorGroup;
        if (r < nr) a.P[(size_t)j * a.L + l0 + r] = out[i];
    }
}

template <int TH>
__global__ __launch_bounds__(kPhasorThreads) void k_phasor(PhasorArgs a) {
    phasor_body<TH>(a, blockIdx.x);
}
template <int TH>
__global__ __launch_bounds__(kPhasorThreads) void k_phasor_grouped(Group<PhasorArgs> g) {
    persistent_loop(g, [](const PhasorArgs& a, int bx, int) { phasor_body<TH>(a, bx); });
}


template <typename K>
static int persistent_grid(K kernel, int threads, size_t sh, int total) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, sh) != hipSuccess) per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    const int g = (per_cu > 0 ? per_cu : 1) * cus;
    return g < total ? g : total;
}

template <typename K, typename G>
static hipError_t launch_grouped(K kernel, const G& g, int threads, size_t sh, hipStream_t s) {
    if (g.total <= 0) return hipSuccess;
    if (sh > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e != hipSuccess) return e;
    }
    const int grid = g.mode == kFlat ? g.total : persistent_grid(kernel, threads, sh, g.total);
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), sh, s, g);
    return hipGetLastError();
}

hipError_t launch_phasor(const PhasorArgs& a, hipStream_t s) {
    const int TH = a.T / 2;
    dim3 grid((a.L + kPhasorGroup - 1) / kPhasorGroup);
    size_t sh = (size_t)(TH + a.F * kPhasorGroup) * sizeof(float2);
    switch (TH) {
#define NURSD_PH(n)                                                                          \
    case n:                                                                                  \
        if (sh > 65536) {                                                                    \
            hipError_t e = hipFuncSetAttribute((const void*)k_phasor<n>,                     \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh); \
            if (e != hipSuccess) return e;                                                   \
        }                                                                                    \
        hipLaunchKernelGGL(k_phasor<n>, grid, dim3(kPhasorThreads), sh, s, a);               \
        break;
        NURSD_PH(128) NURSD_PH(256) NURSD_PH(512) NURSD_PH(1024) NURSD_PH(2048) NURSD_PH(4096)
#undef NURSD_PH
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_phasor_grouped(int T, int F_max, const Group<PhasorArgs>& g, hipStream_t s) {
    const size_t sh = (size_t)(T / 2 + F_max * kPhasorGroup) * sizeof(float2);
    switch (T / 2) {
#define NURSD_PG(n) \
    case n: return launch_grouped(k_phasor_grouped<n>, g, kPhasorThreads, sh, s);
        NURSD_PG(128) NURSD_PG(256) NURSD_PG(512) NURSD_PG(1024) NURSD_PG(2048) NURSD_PG(4096)
#undef NURSD_PG
        default: return hipErrorInvalidValue;
    }
}

int phasor_group() { return kPhasorGroup; }

}  // namespace nursd
