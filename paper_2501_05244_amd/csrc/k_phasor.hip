// Step 1: temporal phasor transform.
//
// Per relay sample l and kept DFT bin b:
//   P[b][l] = w(f_b) e^{-j 2 pi f_b t0} sum_t H[l][t] e^{-j 2 pi b t / T}
// (the phasor-field response of eq. PF_Response with the Gaussian
// band-pass illumination of eq. PFPacket_Omega_Supp).  The real T-point
// transform is one T/2-point complex transform Z of z[t] = h[2t] + j h[2t+1],
// split as X[b] = E[b] + e^{-j 2 pi b/T} O[b] with
// E = (Z[b] + conj Z[T/2-b]) / 2 and O = (Z[b] - conj Z[T/2-b]) / (2j).
// HBM-bound: each histogram is read once, F values written per sample.
//
// For T = 2048 and 4096 one wavefront transforms one histogram at a time in
// registers: Z is split once more into the N = T/4-point transforms A of the
// even and B of the odd z samples (Z[n] = A[n mod N] + W_{T/2}^n B[n mod N]),
// each a register-resident wave FFT, and the next histogram's loads are in
// flight meanwhile.  Since X is linear in Z[b] and conj Z[T/2-b],
//   X[b] = (al A[b] + be conj A[-b]) + W_{T/2}^b (al B[b] + be conj B[-b])
// with al = (1 - j t_b) / 2, be = (1 + j t_b) / 2, t_b = e^{-j 2 pi b/T} and
// indices mod N, so the A and B halves are gathered one after the other
// through the same LDS scratch.  Other T (and histograms that are not
// 16-byte aligned) use a block-level LDS transform per histogram.
#include "fft.hpp"
#include "kernels.hpp"
#include "persistent.hpp"
#include "wavefft.hpp"

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

constexpr int kPhasorWaves = kPhasorThreads / 64;

// LDS of the wavefront variant: twiddles [N], staged outputs [F][group],
// per-wave scratch.
template <int TH>
constexpr size_t phasor_wave_lds(int F) {
    return (size_t)(TH / 2 + F * kPhasorGroup + kPhasorWaves * WaveFFT<TH / 2>::SCR) * sizeof(float2);
}

template <int TH>
__device__ __forceinline__ void phasor_wave_body(const PhasorArgs& a, int bx) {
    constexpr int N = TH / 2;
    using W = WaveFFT<N>;
    static_assert(W::LPW == 1, "one transform per wavefront");
    constexpr int E = W::E;
    extern __shared__ float2 smem[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    float2* tws = smem;                                      // [N]
    float2* out = smem + N;                                  // [F][kPhasorGroup]
    float2* scr = out + a.F * kPhasorGroup + wave * W::SCR;  // this wave's scratch
    for (int i = tid; i < N; i += kPhasorThreads) tws[i] = a.tw[2 * i];
    __syncthreads();
    const int l0 = bx * kPhasorGroup;
    const int nr = min(kPhasorGroup, a.L - l0);
    // histogram r of the group -> z[2m], z[2m+1] for m = lane + 64 e
    float4 pre[E];
    auto load = [&](int r) {
        const float4* row = reinterpret_cast<const float4*>(a.hist + (size_t)(l0 + r) * a.T);
#pragma unroll
        for (int e = 0; e < E; ++e) pre[e] = row[lane + 64 * e];
    };
    // The spectrum sits in the scratch at a swizzled index: bits 5 and up of
    // k (one bit for N = 512, two for N = 1024) are XORed into bits 2 and up,
    // so the 32 lanes of each half-wave of a spill store hit distinct bank
    // pairs (the natural index puts 2 or 4 of them on one pair).  The map
    // permutes each aligned block of 32 entries: the scratch size is unchanged.
    auto sw = [](int k) { return k ^ (((k >> 5) & (E / 4 - 1)) << 2); };
    // spectrum half h (0: A, 1: B) gathered into the staged outputs of r
    auto gather = [&](int half, int r) {
        for (int j = lane; j < a.F; j += 64) {
            const int b = a.bins[j];
            const float2 t = a.tb[j];
            const float2 u1 = scr[sw(b & (N - 1))];
            const float2 u2 = cconj(scr[sw((N - b) & (N - 1))]);
            // al u1 + be u2 with al = (1 - j t)/2, be = (1 + j t)/2
            const float2 jt = make_float2(-t.y, t.x);
            float2 x = cscale(cadd(cadd(u1, u2), cmul(jt, csub(u2, u1))), 0.5f);
            x = cmul(a.wt[j], x);
            if (half == 0) {
                out[j * kPhasorGroup + r] = x;
            } else {
                const float2 w2 = cmul(t, t);                   // W_{T/2}^b
                out[j * kPhasorGroup + r] = cadd(out[j * kPhasorGroup + r], cmul(w2, x));
            }
        }
    };
    // natural-order spectrum of a wave FFT into the scratch
    auto spill = [&](const float2* v) {
#pragma unroll
        for (int h = 0; h < W::GPL; ++h)
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                int q;
                scr[sw(W::perm_k(lane, h, d, q))] = v[h * 8 + d];
            }
    };
    int r = wave;
    if (r < nr) load(r);
    for (; r < nr; r += kPhasorWaves) {                      // wave-uniform
        float2 va[E], vb[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            va[e] = make_float2(pre[e].x, pre[e].y);
            vb[e] = make_float2(pre[e].z, pre[e].w);
        }
        if (r + kPhasorWaves < nr) load(r + kPhasorWaves);
        W::template nat_to_perm<false>(va, scr, tws, lane);
        spill(va);
        NURSD_WAVE_SYNC();
        gather(0, r);
        NURSD_WAVE_SYNC();
        W::template nat_to_perm<false>(vb, scr, tws, lane);
        spill(vb);
        NURSD_WAVE_SYNC();
        gather(1, r);
        NURSD_WAVE_SYNC();
    }
    __syncthreads();
    for (int i = tid; i < a.F * kPhasorGroup; i += kPhasorThreads) {
        const int j = i / kPhasorGroup, rr = i % kPhasorGroup;
        if (rr < nr) a.P[(size_t)j * a.L + l0 + rr] = out[i];
    }
}

// The wavefront variant needs rows of whole float4 (T of 2048 or 4096 and a
// 16-byte aligned histogram).
template <int TH>
__device__ __forceinline__ bool phasor_wave_ok(const PhasorArgs& a) {
    return TH >= 1024 && TH <= 2048 && (reinterpret_cast<uintptr_t>(a.hist) & 15) == 0;
}

template <int TH>
__global__ __launch_bounds__(kPhasorThreads) void k_phasor(PhasorArgs a) {
    if constexpr (TH >= 1024 && TH <= 2048) {
        if (phasor_wave_ok<TH>(a)) {
            phasor_wave_body<TH>(a, blockIdx.x);
            return;
        }
    }
    phasor_body<TH>(a, blockIdx.x);
}
template <int TH>
__global__ __launch_bounds__(kPhasorThreads) void k_phasor_grouped(Group<PhasorArgs> g) {
    persistent_loop(g, [](const PhasorArgs& a, int bx, int) {
        if constexpr (TH >= 1024 && TH <= 2048) {
            if (phasor_wave_ok<TH>(a)) {
                phasor_wave_body<TH>(a, bx);
                return;
            }
        }
        phasor_body<TH>(a, bx);
    });
}

template <int TH>
static size_t phasor_lds(int F) {
    const size_t blockwise = (size_t)(TH + F * kPhasorGroup) * sizeof(float2);
    if constexpr (TH >= 1024 && TH <= 2048) {
        const size_t wave = phasor_wave_lds<TH>(F);
        return wave > blockwise ? wave : blockwise;
    }
    return blockwise;
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
    switch (TH) {
#define NURSD_PH(n)                                                                          \
    case n: {                                                                                \
        const size_t sh = phasor_lds<n>(a.F);                                                \
        if (sh > 65536) {                                                                    \
            hipError_t e = hipFuncSetAttribute((const void*)k_phasor<n>,                     \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh); \
            if (e != hipSuccess) return e;                                                   \
        }                                                                                    \
        hipLaunchKernelGGL(k_phasor<n>, grid, dim3(kPhasorThreads), sh, s, a);               \
        break;                                                                               \
    }
        NURSD_PH(128) NURSD_PH(256) NURSD_PH(512) NURSD_PH(1024) NURSD_PH(2048) NURSD_PH(4096)
#undef NURSD_PH
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_phasor_grouped(int T, int F_max, const Group<PhasorArgs>& g, hipStream_t s) {
    switch (T / 2) {
#define NURSD_PG(n) \
    case n: return launch_grouped(k_phasor_grouped<n>, g, kPhasorThreads, phasor_lds<n>(F_max), s);
        NURSD_PG(128) NURSD_PG(256) NURSD_PG(512) NURSD_PG(1024) NURSD_PG(2048) NURSD_PG(4096)
#undef NURSD_PG
        default: return hipErrorInvalidValue;
    }
}

int phasor_group() { return kPhasorGroup; }

}  // namespace nursd
