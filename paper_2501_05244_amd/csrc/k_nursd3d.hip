// Stage 1 of the 3D NURSD (eq. 3D_NURSD, with the 3D RSD kernel of
// eq. 3d_rsd): non-planar relay samples (x_l, y_l, z_l) to the field on the
// intermediate plane z0.  The 3D type-1 NUFFT onto I_M^2 x I_Mz (depth frame
// centred on z0, pitch dz), times the 3D DFT of the sampled kernel, inverse
// 3D DFT read at z0, is regrouped along depth: with the relay's depth weights
//   W_p(l) = Mz^-1 sum_{kz in I_Mz} e^{-j kz (z~_l + 2 pi p / Mz)},
//   z~_l = 2 pi (z_l - z0) / (Mz dz)   (host, FP64),
// the plane's spectrum is
//   U0[k] = sum_{p in I_Mz} Ghat(p dz)[k] * NUFFT2{P_l W_p(l)}[k],
// where Ghat(d) is the 2D DFT of the kernel samples at depth offset d.
//   k_modulate:       Q[p][b][l] = P[b][l] W_p(l)  (then the 2D type-1 steps)
//   k_stage1_reduce:  per kx line, Ghat(p dz) along y from the quadrant rows
//                     (cosine transform, as the column pass does), times the
//                     spectra rows at +kx and -kx, summed over p.
#include "kernels.hpp"
#include "wavefft.hpp"

namespace nursd {

__global__ __launch_bounds__(256) void k_modulate(ModulateArgs a) {
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= a.L) return;
    const int i = blockIdx.y;                 // p * nb + b
    const int pz = i / a.nb, b = i % a.nb;
    a.Q[(size_t)i * a.L + l] = cmul(a.P[(size_t)(a.b0 + b) * a.L + l], a.W[(size_t)pz * a.L + l]);
}

hipError_t launch_modulate(const ModulateArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_modulate, dim3((a.L + 255) / 256, a.Mz * a.nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Four waves per block: measured 12 % faster than eight for the reduction
// (more blocks per CU over the (M/2+1)/LPW lines of a frequency).
constexpr int kS1Waves = 4;

template <int M>
__global__ __launch_bounds__(kS1Waves * 64) void k_stage1_reduce(Stage1Args a) {
    using F = WaveFFT<M>;
    constexpr int H = M / 2, E = F::E, LPW = F::LPW;
    extern __shared__ float2 sm[];      // [kS1Waves][SCR], then twiddles [M]
    float2* tws = sm + kS1Waves * F::SCR;
    for (int i = threadIdx.x; i < M; i += kS1Waves * 64) tws[i] = a.tw[i];
    __syncthreads();
    const int bl = blockIdx.y;                // frequency b0 + bl
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kx0 = (blockIdx.x * kS1Waves + wave) * LPW;
    if (kx0 > H) return;                      // wave-uniform; no block barriers below
    float2* scr = sm + wave * F::SCR;
    float2 ap[F::NV], am[F::NV];
#pragma unroll
    for (int i = 0; i < F::NV; ++i) ap[i] = am[i] = make_float2(0.f, 0.f);
    for (int pz = 0; pz < a.Mz; ++pz) {
        const float2* Bt = a.Bt + (size_t)(bl * a.Mz + pz) * (H + 1) * a.BS;
        float2 g[F::NV];
#pragma unroll
        for (int q = 0; q < LPW; ++q) {
            const int kx = kx0 + q;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int n = lane + 64 * e;
                g[q * E + e] = kx <= H ? Bt[(size_t)kx * a.BS + (n <= H ? n : M - n)] : make_float2(0.f, 0.f);
            }
        }
        F::template nat_to_perm<false>(g, scr, tws, lane);
        const float2* Ub = a.Ut + (size_t)(pz * a.g.nb + bl) * M * M;
#pragma unroll
        for (int h = 0; h < F::GPL; ++h)
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                int q;
                const int k = F::perm_k(lane, h, d, q);
                const int kx = kx0 + q;
                if (kx > H) continue;
                ap[h * 8 + d] = cadd(ap[h * 8 + d], cmul(Ub[(size_t)kx * M + k], g[h * 8 + d]));
                am[h * 8 + d] = cadd(am[h * 8 + d], cmul(Ub[(size_t)((M - kx) & (M - 1)) * M + k], g[h * 8 + d]));
            }
    }
    float2* U0 = a.U0 + (size_t)(a.g.b0 + bl) * M * M;
#pragma unroll
    for (int h = 0; h < F::GPL; ++h)
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            int q;
            const int k = F::perm_k(lane, h, d, q);
            const int kx = kx0 + q;
            if (kx > H) continue;
            const int sm_ = (M - kx) & (M - 1);
            U0[(size_t)kx * M + k] = ap[h * 8 + d];
            if (sm_ != kx) U0[(size_t)sm_ * M + k] = am[h * 8 + d];
        }
}

hipError_t launch_stage1_reduce(const Stage1Args& a, hipStream_t s) {
    switch (a.M) {
#define NURSD_S1(MM)                                                                                     \
    case MM: {                                                                                           \
        using F = WaveFFT<MM>;                                                                           \
        constexpr int LB = kS1Waves * F::LPW;                                                            \
        hipLaunchKernelGGL(k_stage1_reduce<MM>, dim3((MM / 2 + 1 + LB - 1) / LB, a.g.nb), dim3(kS1Waves * 64), \
                           (size_t)(kS1Waves * F::SCR + MM) * sizeof(float2), s, a);                     \
        return hipGetLastError();                                                                        \
    }
        NURSD_S1(64) NURSD_S1(128) NURSD_S1(256) NURSD_S1(512) NURSD_S1(1024)
#undef NURSD_S1
        default: return hipErrorInvalidValue;
    }
}

}  // namespace nursd
