// Step 5 for arbitrary voxels (eq. NURSD2 / eq. NURSD3): type-2 NUFFT of
// X = U_b * Ghat_{b,z} at each plane's voxel list,
//   F(x_v) = M^-2 sum_{k in I_M^2} U_b[k] Ghat[k] e^{+j k.x~_v},
// by the reverse of the type-1 steps (NUFFT section): deconvolve by the
// kernel's Fourier coefficients, zero-pad to the oversampled grid, inverse
// FFT, interpolate with the same exponential-of-semicircle kernel.
//   k_type2_cols: Ghat along y (cosine transform of the quadrant rows), times
//                 U[+kx], U[-kx] and the x and y deconvolution factors
//                 (with the (-1)^k of the centred fine grid), zero-padded
//                 Mf-point inverse FFT along y -> T2[p][kx][jy].
//   k_type2_band: per band of kType2RowBand fine rows, Mf-point inverse FFT
//                 along x of the zero-padded rows, kept in LDS, and the w x w
//                 interpolation of every voxel whose taps reach the band,
//                 restricted to those rows -> partial sums per (frequency,
//                 voxel-band entry).  The fine grid is never stored.
//   k_type2_gather: per voxel, its one or two partial sums of every frequency
//                 of the chunk, illumination phase (advanced by a per-voxel
//                 step factor over the evenly spaced frequencies of the
//                 chunk), accumulation.
#include "kernels.hpp"
#include "wavefft.hpp"

namespace nursd {

__device__ __forceinline__ float es_w(float z, float beta) {
    const float t = fmaxf(1.0f - z * z, 0.0f);
    return __expf(beta * (sqrtf(t) - 1.0f));
}

constexpr int kT2Waves = 4;
constexpr int kT2RowWaves = kType2RowBand;

template <int M>
__global__ __launch_bounds__(kT2Waves * 64) void k_type2_cols(Type2Args a) {
    using F = WaveFFT<M>;
    using G = WaveFFT<2 * M>;
    constexpr int H = M / 2, MF = 2 * M, E = F::E, EG = G::E;
    static_assert(F::LPW == 1, "type-2 output needs M >= 512 per wave line");
    constexpr int SCRP = G::SCR + 1;
    extern __shared__ float2 sm[];          // [kT2Waves][SCRP], twiddles M, twiddles MF
    float2* tws_m = sm + kT2Waves * SCRP;
    float2* tws_f = tws_m + M;
    for (int i = threadIdx.x; i < M; i += kT2Waves * 64) tws_m[i] = a.tw_m[i];
    for (int i = threadIdx.x; i < MF; i += kT2Waves * 64) tws_f[i] = a.tw_f[i];
    __syncthreads();
    // each XCD takes a contiguous run of (plane, kx block) items: the planes
    // of one frequency share its spectrum rows, which then stay in that L2
    const int vb = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int bxx = vb % gridDim.x, p = vb / gridDim.x;
    const int b = a.g.b0 + p / a.g.nzc;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kx = bxx * kT2Waves + wave;
    if (kx > H) return;
    float2* scr = sm + wave * SCRP;
    const float2* Bt = a.Bt + (size_t)p * (H + 1) * a.BS;
    float2 g[F::NV];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int n = lane + 64 * e;
        g[e] = Bt[(size_t)kx * a.BS + (n <= H ? n : M - n)];
    }
    F::template nat_to_perm<false>(g, scr, tws_m, lane);
    const float2* Ub = a.U + (size_t)b * M * M;
    float2* T2 = a.T2 + (size_t)p * M * MF;
    // only the fine rows the row pass reads are stored
    const int iz = a.g.z0 + p % a.g.nzc;
    const int lo = a.row_lo[iz], hi = a.row_hi[iz];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int s = side ? ((M - kx) & (M - 1)) : kx;
        if (side && s == kx) break;
        const float dx = a.dec[s];
        // product in FFT order of M, staged into the zero-padded natural MF line
        NURSD_WAVE_SYNC();
        for (int i = lane; i < MF; i += 64) scr[i] = make_float2(0.f, 0.f);
        NURSD_WAVE_SYNC();
#pragma unroll
        for (int h = 0; h < F::GPL; ++h)
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                int q;
                const int k = F::perm_k(lane, h, d, q);      // ky mod M
                const int kf = k < H ? k : k + (MF - M);     // ky mod MF
                scr[kf] = cscale(cmul(Ub[(size_t)s * M + k], g[h * 8 + d]), dx * a.dec[k]);
            }
        NURSD_WAVE_SYNC();
        float2 v[G::NV];
#pragma unroll
        for (int e = 0; e < EG; ++e) v[e] = scr[lane + 64 * e];
        G::template nat_to_perm<true>(v, scr, tws_f, lane);
#pragma unroll
        for (int h = 0; h < G::GPL; ++h)
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                int q;
                const int jy = G::perm_k(lane, h, d, q);
                if (type2_row_stored(jy, lo, hi, MF)) T2[(size_t)s * MF + jy] = v[h * 8 + d];
            }
    }
}

__device__ __forceinline__ double dist3d(double x, double y, double z) {
    const double d2 = x * x + y * y + z * z;
    float inv;
    return sqrt_f64(d2, &inv);
}

// Fine-grid position of voxel v on plane iz: first tap (ix0, iy0), offsets of
// the voxel from them (fx, fy) in fine cells, and its w x w kernel weights.
__device__ __forceinline__ void voxel_taps(const Type2Args& a, int v, int iz, int& ix0, int& iy0, float* wx,
                                           float* wy) {
    const int MF = a.Mf;
    const double x = a.voxel_xy[2 * v], y = a.voxel_xy[2 * v + 1];
    const double hw = 0.5 * a.w;
    // plane pitch: the frame pitch, or dx / alpha on a scaled plane
    const double px = a.g.pitch_x ? a.g.pitch_x[iz] : a.g.dx;
    const double py = a.g.pitch_y ? a.g.pitch_y[iz] : a.g.dy;
    const double tx = (x - a.cx) / px * 2.0 + MF / 2;
    const double ty = (y - a.cy) / py * 2.0 + MF / 2;
    ix0 = (int)ceil(tx - hw);
    iy0 = (int)ceil(ty - hw);
    const float fx = (float)(tx - ix0), fy = (float)(ty - iy0);
    const float ihw = (float)(1.0 / hw);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        wx[i] = i < a.w ? es_w(((float)i - fx) * ihw, a.beta) : 0.f;
        wy[i] = i < a.w ? es_w(((float)i - fy) * ihw, a.beta) : 0.f;
    }
}

// One workgroup per band of RB fine rows of one (frequency, plane): inverse
// FFT along x of the band's zero-padded rows, kept in LDS, then the w x w
// interpolation of every voxel whose taps reach the band, restricted to the
// band's rows; the partial sums go to part[frequency][entry].
template <int M>
__global__ __launch_bounds__(kT2RowWaves * 64) void k_type2_band(Type2Args a) {
    using G = WaveFFT<2 * M>;
    constexpr int H = M / 2, MF = 2 * M, EG = G::E;
    constexpr int TP = M + 1;               // tile row: the M data values of a line
    constexpr int RB = kT2RowWaves;
    static_assert(TP <= G::SCR && MF <= G::SCR && H % 64 == 0, "tile layout");
    // The block's RB rows are staged compactly (the zero padding is never
    // stored), read into registers, and the tile is then reused as the waves'
    // FFT scratch and finally holds the transformed rows: 80 KB at M = 512, so
    // two blocks share a CU.
    extern __shared__ float2 sm[];          // tile [RB][TP] / scratch and rows [RB][SCR], twiddles MF
    float2* tws = sm + RB * G::SCR;
    for (int i = threadIdx.x; i < MF; i += kT2RowWaves * 64) tws[i] = a.tw_f[i];
    // neighbouring bands of a plane (which share the cache lines of the
    // column outputs they read) run on the same XCD
    const int vb = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int p = vb / gridDim.x;
    const int band = vb % gridDim.x;
    const int zl = p % a.g.nzc, bl = p / a.g.nzc;
    const int iz = a.g.z0 + zl;
    const int jy0 = a.row_lo[iz] + band * RB;
    if (jy0 > a.row_hi[iz]) return;         // block-uniform
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const float2* T2 = a.T2 + (size_t)p * M * MF;
    for (int i = threadIdx.x; i < M * RB; i += kT2RowWaves * 64) {
        const int kx = i / RB, j = i % RB;
        const int jy = (jy0 + j) & (MF - 1);
        sm[j * TP + kx] = T2[(size_t)kx * MF + jy];
    }
    __syncthreads();
    // natural zero-padded line: kx < H at n = kx, kx >= H at n = kx + MF - M
    float2 v[G::NV];
#pragma unroll
    for (int e = 0; e < EG; ++e) {
        const int n = lane + 64 * e;
        if (64 * e < H) v[e] = sm[wave * TP + n];
        else if (64 * e >= MF - H) v[e] = sm[wave * TP + n - (MF - M)];
        else v[e] = make_float2(0.f, 0.f);
    }
    __syncthreads();                        // all rows read: the tile becomes scratch
    float2* scr = sm + wave * G::SCR;
    G::template nat_to_perm<true>(v, scr, tws, lane);
    // row jy0 + wave of the fine grid, natural column order, in this wave's region
#pragma unroll
    for (int h = 0; h < G::GPL; ++h)
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            int q;
            scr[G::perm_k(lane, h, d, q)] = v[h * 8 + d];
        }
    __syncthreads();
    const int bi = a.plane_band[iz] + band;
    const int e1 = a.band_ptr[bi + 1];
    float2* part = a.part + (size_t)bl * a.n_lent;
    for (int e = a.band_ptr[bi] + threadIdx.x; e < e1; e += kT2RowWaves * 64) {
        int ix0, iy0;
        float wx[8], wy[8];
        voxel_taps(a, a.ent_vox[e], iz, ix0, iy0, wx, wy);
        int col[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) col[i] = (ix0 + i) & (MF - 1);
        float2 sum = make_float2(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (j >= a.w) break;
            const int lr = (iy0 + j - jy0) & (MF - 1);       // row within the band
            if (lr >= RB) continue;
            const float2* row = sm + lr * G::SCR;
            float2 r = make_float2(0.f, 0.f);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                if (i >= a.w) break;
                const float2 gv = row[col[i]];
                r.x = fmaf(wx[i], gv.x, r.x);
                r.y = fmaf(wx[i], gv.y, r.y);
            }
            sum.x = fmaf(wy[j], r.x, sum.x);
            sum.y = fmaf(wy[j], r.y, sum.y);
        }
        part[e] = sum;
    }
}

constexpr int kGatherThreads = 256;

// Per voxel: the partial sums of its one or two bands for every frequency of
// the chunk, times the illumination phase (advanced by a per-voxel step factor
// over the evenly spaced frequencies of the chunk), accumulated into V / I.
__global__ __launch_bounds__(kGatherThreads) void k_type2_gather(Type2Args a) {
    const int zl = blockIdx.y;
    const int iz = a.g.z0 + zl;
    const int v = a.plane_ptr[iz] + blockIdx.x * kGatherThreads + threadIdx.x;
    if (v >= a.plane_ptr[iz + 1]) return;
    const int e0 = a.vox_ent[2 * v], e1 = a.vox_ent[2 * v + 1];
    float2 acc = make_float2(0.f, 0.f);
    if (!a.first) {
        if (a.coherent) acc = a.V[v];
        else acc.x = a.I[v];
    }
    float2 ph = make_float2(1.f, 0.f), st = make_float2(1.f, 0.f);
    if (a.coherent) {
        const double x = a.voxel_xy[2 * v], y = a.voxel_xy[2 * v + 1];
        const double dd = dist3d(x - a.xp0, y - a.xp1, a.g.z[iz] - a.xp2);
        const double cyc0 = dd * (a.g.f[a.g.b0] / kC), cyc1 = dd * (a.g.df / kC);
        float sn, cs;
        sincos_cycles((float)(cyc0 - rint(cyc0)), &sn, &cs);
        ph = make_float2(cs, sn);
        sincos_cycles((float)(cyc1 - rint(cyc1)), &sn, &cs);
        st = make_float2(cs, sn);
    }
    for (int bl = 0; bl < a.g.nb; ++bl) {
        const float2* part = a.part + (size_t)bl * a.n_lent;
        float2 s = part[e0];
        if (e1 >= 0) s = cadd(s, part[e1]);
        if (a.coherent) {
            acc = cadd(acc, cmul(ph, s));
            ph = cmul(ph, st);
        } else {
            acc.x += sqrtf(s.x * s.x + s.y * s.y);
        }
    }
    if (a.coherent) {
        a.V[v] = acc;
        if (a.last && a.I) a.I[v] = sqrtf(acc.x * acc.x + acc.y * acc.y);
    } else {
        a.I[v] = acc.x;
    }
}

template <typename Args>
static hipError_t launch_t2(void (*k)(Args), dim3 grid, int threads, size_t sh, hipStream_t s, const Args& a) {
    if (sh > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, grid, dim3(threads), sh, s, a);
    return hipGetLastError();
}

template <int M>
static hipError_t type2_fine_impl(const Type2Args& a, hipStream_t s) {
    using G = WaveFFT<2 * M>;
    const int planes = a.g.nb * a.g.nzc;
    hipError_t e = launch_t2(k_type2_band<M>, dim3((2 * M + kT2RowWaves - 1) / kT2RowWaves, planes),
                             kT2RowWaves * 64, (size_t)(kT2RowWaves * G::SCR + 2 * M) * sizeof(float2), s, a);
    if (e != hipSuccess) return e;
    return launch_t2(k_type2_gather, dim3((a.max_vox + kGatherThreads - 1) / kGatherThreads, a.g.nzc),
                     kGatherThreads, 0, s, a);
}

template <int M>
static hipError_t type2_impl(const Type2Args& a, hipStream_t s) {
    using G = WaveFFT<2 * M>;
    const int planes = a.g.nb * a.g.nzc;
    hipError_t e = launch_t2(k_type2_cols<M>, dim3((M / 2 + 1 + kT2Waves - 1) / kT2Waves, planes), kT2Waves * 64,
                             (size_t)(kT2Waves * (G::SCR + 1) + M + 2 * M) * sizeof(float2), s, a);
    if (e != hipSuccess) return e;
    return type2_fine_impl<M>(a, s);
}

hipError_t launch_type2(const Type2Args& a, hipStream_t s) {
    if (!a.g.uni) return hipErrorInvalidValue;     // phases advance by a fixed step
    switch (a.M) {
        case 512: return type2_impl<512>(a, s);
        case 1024: return type2_impl<1024>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_type2_fine(const Type2Args& a, hipStream_t s) {
    if (!a.g.uni) return hipErrorInvalidValue;     // phases advance by a fixed step
    switch (a.M) {
        case 512: return type2_fine_impl<512>(a, s);
        case 1024: return type2_fine_impl<1024>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace nursd
