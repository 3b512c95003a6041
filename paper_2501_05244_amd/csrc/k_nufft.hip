// Steps 2-3: type-1 NUFFT of the phasors of one frequency onto M x M modes
// (the three steps of the NUFFT section: spread with a blur kernel onto an
// oversampled grid, FFT, deconvolve by the kernel's Fourier coefficients).
//
// Blur kernel: exponential of semicircle psi(z) = exp(beta (sqrt(1 - z^2) - 1)),
// |z| <= 1, over w fine cells; oversampling sigma = 2 (fine grid Mf = 2M).
//
// k_spread_xfft: one workgroup owns a band of BR fine rows (all Mf columns)
// of NF frequencies in LDS.  Relay samples are pre-binned per band and
// sorted by x; each wavefront owns a disjoint range of columns (split so the
// waves' sample counts balance) and walks the samples overlapping it, one
// sample per step, its lanes spread over (tap column, frequency and band
// row) so the x kernel weight of a sample is computed once for all its
// copies.  Every LDS cell is updated by one wave in a fixed order: no
// atomics, bitwise reproducible.  Each band row is then transformed along x
// (512- and 1024-point rows by one wavefront each in registers, with the row
// itself as exchange scratch; other sizes by the block-level LDS transform)
// and only the M kept modes are written, scaled by the x deconvolution
// factor, band-major ([frequency][band][mode][band row]) so each block writes
// contiguous runs.
// k_fine_y / k_fine_y_wave: FFT along y of each kept kx column, keep M modes,
// deconvolve in y.
#include "fft.hpp"
#include "kernels.hpp"
#include "persistent.hpp"
#include "wavefft.hpp"

namespace nursd {

constexpr int kSpreadThreads = 1024;
// LDS row stride of a band: rows of 512 or 1024 points are transformed along
// x by one wavefront each and double as its exchange scratch (the wave
// transform's padded tiles, (MF / 64) * 8 * RP cells); 8 further cells put
// the rows of one sample's step on different banks.
constexpr int spread_row_stride(int MF) { return (MF >= 512 && MF <= 1024 ? MF / 64 * 8 * NURSD_WFFT_RP : MF) + 8; }
template <int MF>
constexpr int spread_row_stride() { return spread_row_stride(MF); }

// psi(z) = exp(beta (sqrt(1 - z^2) - 1)) with the hardware square root and
// base-2 exponential (beta_log2e = beta / ln 2).
__device__ __forceinline__ float es_kernel(float z, float beta_log2e) {
    const float t = fmaxf(1.0f - z * z, 0.0f);
    return __builtin_amdgcn_exp2f(beta_log2e * (__builtin_amdgcn_sqrtf(t) - 1.0f));
}

__device__ __forceinline__ float lane_f(float v, int j) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

template <int MF, int kBandRows = spread_band_rows(MF), int NF = spread_freqs(MF)>
__device__ __forceinline__ void spread_xfft_body(const SpreadArgs& a, int bx, int by) {
    constexpr int LDT = spread_row_stride<MF>();
    extern __shared__ float2 tile[];   // [NF][kBandRows][LDT]
    const int band = bx;
    const int fa = a.b0 + by * NF;                    // first frequency of the block
    const int nf = min(NF, a.b0 + a.nb - fa);
    const int tid = threadIdx.x;
    const int e0 = a.band_ptr[band], e1 = a.band_ptr[band + 1];
    const int M = a.M;
    const int y0 = band * kBandRows;
    // this band of chunk-local frequency by * NF; a frequency's bands are
    // M * kBandRows apart, so each block writes nf contiguous runs
    float2* T1 = a.T1 + ((size_t)by * NF * (MF / kBandRows) + band) * M * kBandRows;
    constexpr size_t kBands = MF / kBandRows;
    if (e0 == e1) {
        // empty band: its transform is zero
        for (int i = tid; i < nf * M * kBandRows; i += kSpreadThreads) {
            const int f = i / (M * kBandRows), j = i % (M * kBandRows);
            T1[(size_t)f * kBands * M * kBandRows + j] = make_float2(0.f, 0.f);
        }
        return;
    }
    for (int i = tid; i < NF * kBandRows * LDT; i += kSpreadThreads) tile[i] = make_float2(0.f, 0.f);
    __syncthreads();

    static_assert(kSpreadThreads == kSpreadWaves * 64, "one wave per column range");
    const int wave = tid >> 6, lane = tid & 63;
    const int* rng = a.wave_rng + (band * kSpreadWaves + wave) * 4;
    const int c_lo = rng[2], c_hi = rng[3];             // columns owned by this wave
    const float inv_hw = 1.0f / a.half_w;
    const float bl2e = a.beta * 1.4426950408889634f;
    const int w = a.w;
    const int s0 = rng[0], s1 = rng[1];
    const float2* Pb = a.P + (size_t)fa * a.L;
    // Lane (ti, q): tap column ti of tile row n = q + 8 r (round r), the
    // pair (frequency n / BR, band row n % BR).  One step applies one sample
    // to every such pair, so all lanes work when the band's rows lie inside
    // the sample's taps (always for one-row bands).
    constexpr int NQ = NF * kBandRows, RND = (NQ + 7) / 8;
    const int ti = lane & 7, q0 = lane >> 3;
    // 8 * KB entries per round trip: lane (ti, q) fetches entries base + ti +
    // 8 k (k < KB), with the value of its pair's frequency for each round;
    // step j takes entry j from lane (j % 8, q) by a lane permute.
    constexpr int KB = 4;
    for (int base = s0; base < s1; base += 8 * KB) {
        int packed[KB];
        float efx[KB], efy[KB];
        float2 val[KB][RND];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int e = base + ti + 8 * k;
            packed[k] = 0;
            efx[k] = efy[k] = 0.f;
#pragma unroll
            for (int r = 0; r < RND; ++r) val[k][r] = make_float2(0.f, 0.f);
            if (e < s1) {
                const SpreadEntry en = a.ent[e];
                packed[k] = ((int)en.ix0 & 0xffff) | ((int)en.iy0 << 16);
                efx[k] = en.fx;
                efy[k] = en.fy;
                const float wl = a.wts ? a.wts[en.idx] : 1.0f;     // per-sample weight
#pragma unroll
                for (int r = 0; r < RND; ++r) {
                    const int n = q0 + 8 * r, f = n / kBandRows;
                    if (n < NQ && f < nf) val[k][r] = cscale(Pb[(size_t)f * a.L + en.idx], wl);
                }
            }
        }
        const int cnt = min(8 * KB, s1 - base);
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int jn = min(8, cnt - 8 * k);
            for (int jl = 0; jl < jn; ++jl) {
                const int pk = __builtin_amdgcn_readlane(packed[k], jl);
                const float fx = lane_f(efx[k], jl), fy = lane_f(efy[k], jl);
                const int cx = (int)(short)(pk & 0xffff) + ti;
                const int iy0 = pk >> 16;
                const bool x_ok = ti < w && cx >= c_lo && cx < c_hi;
                const float wx = es_kernel(((float)ti - fx) * inv_hw, bl2e);
#pragma unroll
                for (int r = 0; r < RND; ++r) {
                    const int n = q0 + 8 * r;
                    const int tj = y0 + n % kBandRows - iy0;
                    float2 v;
                    v.x = __shfl(val[k][r].x, 8 * q0 + jl);
                    v.y = __shfl(val[k][r].y, 8 * q0 + jl);
                    if (x_ok && n < NQ && tj >= 0 && tj < w) {
                        const float wgt = wx * es_kernel(((float)tj - fy) * inv_hw, bl2e);
                        float2* cell = &tile[n * LDT + cx];
                        float2 c = *cell;
                        c.x = fmaf(v.x, wgt, c.x);
                        c.y = fmaf(v.y, wgt, c.y);
                        *cell = c;
                    }
                }
            }
        }
    }
    __syncthreads();
    if constexpr (MF >= 512 && MF <= 1024) {
        // one row per wavefront: register transform with the row as its
        // exchange scratch (twiddles read through the caches), then the
        // kept modes (the octants d = 0, 1, 6, 7 of MF = 2M) back in place
        using F = WaveFFT<MF>;
        static_assert(F::LPW == 1 && LDT >= F::SCR, "a band row must hold the wave transform's scratch");
        if (wave < NF * kBandRows) {
            float2* row = tile + wave * LDT;
            float2 v[F::NV];
#pragma unroll
            for (int e = 0; e < F::E; ++e) v[e] = row[lane + 64 * e];
            F::template nat_to_perm<false>(v, row, a.tw, lane);
#pragma unroll
            for (int h = 0; h < F::GPL; ++h)
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    if (d >= 2 && d < 6) continue;
                    int q;
                    row[F::perm_k(lane, h, d, q)] = v[h * 8 + d];
                }
        }
        __syncthreads();
    } else {
        fft_lines<MF, kSpreadThreads / (NF * kBandRows), false>(tile, LDT, NF * kBandRows, a.tw);
    }
    // keep modes kx in I_M: FFT index kx mod MF, stored at kx mod M
    for (int i = tid; i < nf * M * kBandRows; i += kSpreadThreads) {
        const int f = i / (M * kBandRows), j = i % (M * kBandRows);
        const int km = j / kBandRows, r = j % kBandRows;           // km = kx mod M
        const int kf = km < M / 2 ? km : km + (MF - M);           // kx mod MF
        const float2 v = tile[(f * kBandRows + r) * LDT + kf];
        T1[(size_t)f * kBands * M * kBandRows + j] = cscale(v, a.decx[km]);
    }
}

constexpr int kFineYThreads = 256;
constexpr int kFineYLines = 4;

// NL lines of MF points per workgroup, NT / NL threads per line (the
// batched variants keep 64 threads per line).  A band of the spreading holds
// the NL lines' values of its br rows contiguously, so the block reads runs
// of NL * br values.  LDS lines are 2 br (at most 16) cells longer than MF:
// the lanes that store one run (l * br + r) then hit distinct banks for the
// launches' NL * br = 16 or 32.
template <int MF>
constexpr int fine_y_ls() { return MF + 16; }      // allocation per line

template <int MF, int NL = kFineYLines, int NT = kFineYThreads>
__device__ __forceinline__ void fine_y_body(const FineYArgs& a, int bx, int by) {
    extern __shared__ float2 buf[];    // [NL][LS]
    const int M = a.M, br = a.br;
    const int LS = MF + 2 * min(br, 8);
    const int kx0 = bx * NL;
    const int fb = by;
    const float2* T1 = a.T1 + (size_t)fb * M * MF + (size_t)kx0 * br;
    float2* U = a.U + (size_t)(a.b0 + fb) * M * M;
    const int tid = threadIdx.x;
    const int run = NL * br;
    for (int i = tid; i < NL * MF; i += NT) {
        const int bnd = i / run, k = i % run;          // band, then (line, row) within the run
        const int l = k / br, c = bnd * br + k % br;
        buf[l * LS + c] = T1[(size_t)bnd * M * br + k];
    }
    __syncthreads();
    fft_lines<MF, NT / NL, false>(buf, LS, NL, a.tw);
    for (int i = tid; i < NL * M; i += NT) {
        const int l = i / M, km = i % M;
        const int kf = km < M / 2 ? km : km + (MF - M);
        U[(size_t)(kx0 + l) * M + km] = cscale(buf[l * LS + kf], a.decy[km]);
    }
}

template <int MF>
__global__ __launch_bounds__(kSpreadThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_spread_xfft(SpreadArgs a) {
    const int v = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    spread_xfft_body<MF>(a, v % gridDim.x, v / gridDim.x);
}
template <int MF, int BR, int NF>
__global__ __launch_bounds__(kSpreadThreads) void k_spread_xfft_grouped(Group<SpreadArgs> g) {
    persistent_loop(g, [](const SpreadArgs& a, int bx, int by) { spread_xfft_body<MF, BR, NF>(a, bx, by); });
}
// Fine y with one register-resident transform per wavefront (one line of
// MF >= 512 points per wave): the block stages its NL lines in LDS as above,
// then each wave transforms its line in registers, using the line's LDS row
// as exchange scratch, and stores the kept modes straight from the permuted
// layout.  Since MF = 2M, the kept modes (k < M/2 or k >= MF - M/2) are the
// slots d = 0, 1, 6, 7 of every 8-point group, so the last radix stage only
// forms those.  No block barrier after the load.
template <int MF, int NL>
constexpr int fine_y_wave_pitch() { return WaveFFT<MF>::SCR + 16; }
template <int MF, int NL>
constexpr size_t fine_y_wave_lds() { return ((size_t)NL * fine_y_wave_pitch<MF, NL>() + MF) * sizeof(float2); }

template <int MF, int NL>
__device__ __forceinline__ void fine_y_wave_body(const FineYArgs& a, int bx, int by) {
    using F = WaveFFT<MF>;
    static_assert(F::LPW == 1 && F::GPL * 8 == F::E, "one line per wavefront");
    extern __shared__ float2 sm[];     // [NL][pitch] lines and exchange scratch, then twiddles [MF]
    float2* tws = sm + NL * fine_y_wave_pitch<MF, NL>();
    const int M = a.M, br = a.br;
    const int LS = F::SCR + 2 * min(br, 8);     // as fine_y_body: lanes of one run on distinct banks
    const int kx0 = bx * NL;
    const int fb = by;
    const float2* T1 = a.T1 + (size_t)fb * M * MF + (size_t)kx0 * br;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int i = tid; i < MF; i += NL * 64) tws[i] = a.tw[i];
    const int run = NL * br;
    for (int i = tid; i < NL * MF; i += NL * 64) {
        const int bnd = i / run, k = i % run;
        const int l = k / br, c = bnd * br + k % br;
        sm[l * LS + c] = T1[(size_t)bnd * M * br + k];
    }
    __syncthreads();
    float2* line = sm + wave * LS;
    float2 v[F::NV];
#pragma unroll
    for (int e = 0; e < F::E; ++e) v[e] = line[lane + 64 * e];
    F::template nat_to_perm<false>(v, line, tws, lane);
    float2* U = a.U + ((size_t)(a.b0 + fb) * M + kx0 + wave) * M;
#pragma unroll
    for (int h = 0; h < F::GPL; ++h)
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            if (d >= 2 && d < 6) continue;
            int q;
            const int k = F::perm_k(lane, h, d, q);
            const int km = d < 2 ? k : k - (MF - M);
            U[km] = cscale(v[h * 8 + d], a.decy[km]);
        }
}

template <int MF, int NL>
__global__ __launch_bounds__(NL * 64) void k_fine_y_wave(FineYArgs a) {
    fine_y_wave_body<MF, NL>(a, blockIdx.x, blockIdx.y);
}

template <int MF, int NL>
__global__ __launch_bounds__(NL * 64) void k_fine_y(FineYArgs a) {
    fine_y_body<MF, NL, NL * 64>(a, blockIdx.x, blockIdx.y);
}
// Batched: the wave transform for 512- and 1024-point lines (the batch's
// scenes all have Mf = 2M), the LDS transform otherwise.
template <int MF, int NL>
__global__ __launch_bounds__(NL * 64) void k_fine_y_grouped(Group<FineYArgs> g) {
    if constexpr (MF == 512 || MF == 1024)
        persistent_loop(g, [](const FineYArgs& a, int bx, int by) { fine_y_wave_body<MF, NL>(a, bx, by); });
    else
        persistent_loop(g, [](const FineYArgs& a, int bx, int by) { fine_y_body<MF, NL, NL * 64>(a, bx, by); });
}
template <int MF, int NL>
constexpr size_t fine_y_grouped_lds() {
    if constexpr (MF == 512 || MF == 1024) return fine_y_wave_lds<MF, NL>();
    else return (size_t)NL * fine_y_ls<MF>() * sizeof(float2);
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

// At most 64 VGPRs (8 waves per SIMD), so that two workgroups of tiles
// within 80 KB share a CU; the register transform of the x pass would
// otherwise take 68.  Workgroups are renumbered so that each XCD takes a
// contiguous run of bands of one frequency group: a sample reaches several
// neighbouring bands, whose reads of its entry and phasors then hit that
// XCD's L2 (10 % faster than the dispatcher's round-robin order).
template <int MF, int BR, int NF>
__global__ __launch_bounds__(kSpreadThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_spread_xfft_var(SpreadArgs a) {
    const int v = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    spread_xfft_body<MF, BR, NF>(a, v % gridDim.x, v / gridDim.x);
}

// A spreading tile (BR rows of NF frequencies, row stride MF + 8) fits LDS
// and the in-LDS transform keeps at least one wavefront per line.
constexpr bool spread_fits(int MF, int BR, int NF) {
    return BR * NF <= 16 && (size_t)BR * NF * spread_row_stride(MF) * sizeof(float2) <= 160 * 1024 && MF / BR >= 2;
}

template <int MF, int BR, int NF>
static hipError_t spread_plain(const SpreadArgs& a, hipStream_t s) {
    if constexpr (spread_fits(MF, BR, NF)) {
        const size_t sh = (size_t)NF * BR * spread_row_stride<MF>() * sizeof(float2);
        void (*k)(SpreadArgs) = nullptr;
        if constexpr (BR == spread_band_rows(MF) && NF == spread_freqs(MF)) k = k_spread_xfft<MF>;
        else k = k_spread_xfft_var<MF, BR, NF>;
        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3(MF / BR, (a.nb + NF - 1) / NF), dim3(kSpreadThreads), sh, s, a);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <int MF>
static hipError_t spread_impl(const SpreadArgs& a, hipStream_t s) {
    switch (a.var) {
        case 0: return spread_plain<MF, spread_band_rows(MF), spread_freqs(MF)>(a, s);
        case spread_var(4, 4): return spread_plain<MF, 4, 4>(a, s);
        case spread_var(2, 8): return spread_plain<MF, 2, 8>(a, s);
        case spread_var(1, 16): return spread_plain<MF, 1, 16>(a, s);
        case spread_var(1, 8): return spread_plain<MF, 1, 8>(a, s);
        case spread_var(8, 2): return spread_plain<MF, 8, 2>(a, s);
        case spread_var(16, 1): return spread_plain<MF, 16, 1>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_spread_xfft(const SpreadArgs& a, hipStream_t s) {
    if (a.Mf != 2 * a.M) return hipErrorInvalidValue;     // kept modes: the octants of sigma = 2
    switch (a.Mf) {
        case 32: return spread_impl<32>(a, s);
        case 64: return spread_impl<64>(a, s);
        case 128: return spread_impl<128>(a, s);
        case 256: return spread_impl<256>(a, s);
        case 512: return spread_impl<512>(a, s);
        case 1024: return spread_impl<1024>(a, s);
        case 2048: return spread_impl<2048>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int MF, int NL>
static hipError_t finey_launch(const FineYArgs& a, hipStream_t s) {
    const size_t sh = (size_t)NL * fine_y_ls<MF>() * sizeof(float2);
    if (sh > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_fine_y<MF, NL>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_fine_y<MF, NL>), dim3(a.M / NL, a.nb), dim3(NL * 64), sh, s, a);
    return hipGetLastError();
}

// Lines per workgroup: enough that the reads of a band are runs of at least
// 16 values (NL * br) where LDS allows.
template <int MF, int NL>
constexpr bool fine_y_fits() { return (size_t)NL * fine_y_ls<MF>() * sizeof(float2) <= 160 * 1024; }

template <int MF, int NL>
static hipError_t finey_wave_launch(const FineYArgs& a, hipStream_t s) {
    constexpr size_t sh = fine_y_wave_lds<MF, NL>();
    static_assert(sh <= 160 * 1024, "fine-y lines must fit LDS");
    if (sh > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_fine_y_wave<MF, NL>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_fine_y_wave<MF, NL>), dim3(a.M / NL, a.nb), dim3(NL * 64), sh, s, a);
    return hipGetLastError();
}

template <int MF>
static hipError_t finey_impl(const FineYArgs& a, hipStream_t s) {
    if constexpr (MF == 512 || MF == 1024) {
        if (a.Mf == 2 * a.M && a.M % 16 == 0) {
            if (a.br <= 1) return finey_wave_launch<MF, 16>(a, s);
            if (a.br <= 2) return finey_wave_launch<MF, 8>(a, s);
            return finey_wave_launch<MF, 4>(a, s);
        }
    }
    if constexpr (fine_y_fits<MF, 16>())
        if (a.br <= 1 && a.M % 16 == 0) return finey_launch<MF, 16>(a, s);
    if constexpr (fine_y_fits<MF, 8>())
        if (a.br <= 2 && a.M % 8 == 0) return finey_launch<MF, 8>(a, s);
    return finey_launch<MF, kFineYLines>(a, s);
}

hipError_t launch_fine_y(const FineYArgs& a, hipStream_t s) {
    switch (a.Mf) {
        case 32: return finey_impl<32>(a, s);
        case 64: return finey_impl<64>(a, s);
        case 128: return finey_impl<128>(a, s);
        case 256: return finey_impl<256>(a, s);
        case 512: return finey_impl<512>(a, s);
        case 1024: return finey_impl<1024>(a, s);
        case 2048: return finey_impl<2048>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int MF, int BR, int NF>
static hipError_t spread_grouped(const Group<SpreadArgs>& g, hipStream_t s) {
    if constexpr (spread_fits(MF, BR, NF)) {
        return launch_grouped(k_spread_xfft_grouped<MF, BR, NF>, g, kSpreadThreads,
                              (size_t)NF * BR * spread_row_stride<MF>() * sizeof(float2), s);
    } else {
        return hipErrorInvalidValue;
    }
}

template <int MF>
static hipError_t spread_grouped_mf(int var, const Group<SpreadArgs>& g, hipStream_t s) {
    switch (var) {
        case 0: return spread_grouped<MF, spread_band_rows(MF), spread_freqs(MF)>(g, s);
        case spread_var(1, 8): return spread_grouped<MF, 1, 8>(g, s);
        case spread_var(1, 16): return spread_grouped<MF, 1, 16>(g, s);
        case spread_var(2, 8): return spread_grouped<MF, 2, 8>(g, s);
        case spread_var(4, 1): return spread_grouped<MF, 4, 1>(g, s);
        case spread_var(4, 2): return spread_grouped<MF, 4, 2>(g, s);
        case spread_var(4, 4): return spread_grouped<MF, 4, 4>(g, s);
        case spread_var(8, 1): return spread_grouped<MF, 8, 1>(g, s);
        case spread_var(8, 2): return spread_grouped<MF, 8, 2>(g, s);
        case spread_var(16, 1): return spread_grouped<MF, 16, 1>(g, s);
        default: return hipErrorInvalidValue;
    }
}

bool spread_var_ok(int Mf, int var) {
    if (Mf < 128 || Mf > 2048 || (Mf & (Mf - 1))) return false;
    if (var == 0) return true;
    const int br = var / 100, nf = var % 100;
    if (!((br == 1 && (nf == 8 || nf == 16)) || (br == 2 && nf == 8) || (br == 4 && (nf == 1 || nf == 2 || nf == 4)) ||
          (br == 8 && (nf == 1 || nf == 2)) || (br == 16 && nf == 1)))
        return false;
    return spread_fits(Mf, br, nf);
}

bool spread_var_plain_ok(int Mf, int var) {
    return var == 0 || ((var == spread_var(4, 4) || var == spread_var(2, 8) || var == spread_var(1, 16) ||
                         var == spread_var(1, 8) || var == spread_var(8, 2) || var == spread_var(16, 1)) &&
                        spread_fits(Mf, var / 100, var % 100) && Mf >= 32 && Mf <= 2048);
}

hipError_t launch_spread_xfft_grouped(int Mf, int var, const Group<SpreadArgs>& g, hipStream_t s) {
    switch (Mf) {
        case 128: return spread_grouped_mf<128>(var, g, s);
        case 256: return spread_grouped_mf<256>(var, g, s);
        case 512: return spread_grouped_mf<512>(var, g, s);
        case 1024: return spread_grouped_mf<1024>(var, g, s);
        case 2048: return spread_grouped_mf<2048>(var, g, s);
        default: return hipErrorInvalidValue;
    }
}

template <int MF>
static hipError_t fine_y_grouped_mf(int lines, const Group<FineYArgs>& g, hipStream_t s) {
    switch (lines) {
#define NURSD_FG(NL) \
    case NL: return launch_grouped(k_fine_y_grouped<MF, NL>, g, NL * 64, fine_y_grouped_lds<MF, NL>(), s);
        NURSD_FG(2) NURSD_FG(4) NURSD_FG(8)
#undef NURSD_FG
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fine_y_grouped(int Mf, int lines, const Group<FineYArgs>& g, hipStream_t s) {
    switch (Mf) {
        case 128: return fine_y_grouped_mf<128>(lines, g, s);
        case 256: return fine_y_grouped_mf<256>(lines, g, s);
        case 512: return fine_y_grouped_mf<512>(lines, g, s);
        case 1024: return fine_y_grouped_mf<1024>(lines, g, s);
        case 2048: return fine_y_grouped_mf<2048>(lines, g, s);
        default: return hipErrorInvalidValue;
    }
}

int fine_y_lines() { return kFineYLines; }

}  // namespace nursd
