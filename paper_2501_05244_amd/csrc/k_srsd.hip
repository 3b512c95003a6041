// Step 6: scaled RSD (eq. SRSD_conv) with the scaled FFT of eq. SFFT and
// its chirp-z derivation (eq. RSD_scale, eq. RSD_scaleconv).
//
// Per frequency, the uniform relay grid u = crop_{N x N}(IDFT_M(U)) is formed
// from the type-1 NUFFT spectrum (fusion for non-uniform acquisition):
//   k_relay_grid_rows: inverse FFT along y of each spectrum row, keep the N
//                      window rows (transposed store [kx][iy]);
//   k_relay_grid_cols: inverse FFT along x, keep the N window columns.
// Per (frequency, plane) with scale alpha:
//   S[k] = sum_{n in I_N^2} u[n] e^{-2 pi j alpha k.n / M},  k in I_M^2,
// separable, each 1D pass by Bluestein's identity
//   alpha k n = alpha/2 (k^2 + n^2 - (k - n)^2):
//   S[k] = e^{-j pi alpha k^2/M} sum_n (u[n] e^{-j pi alpha n^2/M}) e^{+j pi alpha (k-n)^2/M},
// a linear convolution.  The M outputs are split into two halves of M/2, each
// a circular convolution of length M (>= N + M/2 - 1 for N <= M/2 + 1) against
// its own precomputed chirp spectrum; both share the forward FFT of the
// pre-chirped input.  The tables are per plane and built on the host from
// FP64 arguments: the chirp c[m] = e^{-j pi alpha m^2 / M} for m in
// [-M/2, M/2) (the input chirp of n in I_N is c[n]) and the two spectra.
//   k_chirp_rows: Bluestein along x for each of the N rows, times the input
//                 chirp of the y pass (one value per row); store transposed
//                 S1t[p][kx][iy].
//   k_chirp_cols: Bluestein along y for kx and -kx; the output chirp is
//                 folded into the DCT of the kernel sampled at pitch d/alpha
//                 (finished from k_kernel_rows output, even in kx), which both
//                 columns multiply; inverse FFT along y, keep the window.
// The x pass of the inverse transform and the volume formation are the
// uniform-grid k_propagate_rows with per-plane voxel pitch d/alpha.
#include "kernels.hpp"
#include "wavefft.hpp"

namespace nursd {

constexpr int kGridWaves = 8;

// u-pass 1: Tg[b][kx][iy] = sum_ky Us[b][kx][ky] e^{+2 pi j ky (iy - N/2) / M}
template <int M>
__global__ __launch_bounds__(kGridWaves * 64) void k_relay_grid_rows(RelayGridArgs a) {
    using F = WaveFFT<M>;
    constexpr int H = M / 2, E = F::E, LPW = F::LPW;
    extern __shared__ float2 sm[];
    float2* tws = sm + kGridWaves * F::SCR;
    for (int i = threadIdx.x; i < M; i += kGridWaves * 64) tws[i] = a.tw_m[i];
    __syncthreads();
    const int fb = blockIdx.y;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kx0 = (blockIdx.x * kGridWaves + wave) * LPW;
    if (kx0 >= M) return;
    const float2* Ub = a.U + (size_t)(a.b0 + fb) * M * M;
    float2 v[F::NV];
#pragma unroll
    for (int q = 0; q < LPW; ++q)
#pragma unroll
        for (int e = 0; e < E; ++e) v[q * E + e] = Ub[(size_t)(kx0 + q) * M + lane + 64 * e];
    F::template nat_to_perm<true>(v, sm + wave * F::SCR, tws, lane);
    float2* T = a.Tg + (size_t)fb * M * a.N;
#pragma unroll
    for (int h = 0; h < F::GPL; ++h)
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            int q;
            const int k = F::perm_k(lane, h, d, q);
            const int iy = (k < H ? k : k - M) + a.N / 2;
            if (iy >= 0 && iy < a.N) T[(size_t)(kx0 + q) * a.N + iy] = v[h * 8 + d];
        }
}

// u-pass 2: u[b][iy][ix] = sum_kx Tg[b][kx][iy] e^{+2 pi j kx (ix - N/2) / M}
template <int M>
__global__ __launch_bounds__(kGridWaves * 64) void k_relay_grid_cols(RelayGridArgs a) {
    using F = WaveFFT<M>;
    constexpr int H = M / 2, E = F::E, LPW = F::LPW;
    constexpr int SCRP = (F::SCR > LPW * M ? F::SCR : LPW * M) + 1;
    constexpr int RB = kGridWaves * LPW;
    extern __shared__ float2 sm[];
    float2* tws = sm + kGridWaves * SCRP;
    for (int i = threadIdx.x; i < M; i += kGridWaves * 64) tws[i] = a.tw_m[i];
    const int fb = blockIdx.y;
    const int iy0 = blockIdx.x * RB;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int N = a.N;
    const float2* T = a.Tg + (size_t)fb * M * N;
    for (int i = threadIdx.x; i < M * RB; i += kGridWaves * 64) {
        const int s = i / RB, j = i % RB;
        const int iy = iy0 + j;
        sm[(j / LPW) * SCRP + (j % LPW) * M + s] = iy < N ? T[(size_t)s * N + iy] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    float2* rows = sm + wave * SCRP;
    float2 v[F::NV];
#pragma unroll
    for (int q = 0; q < LPW; ++q)
#pragma unroll
        for (int e = 0; e < E; ++e) v[q * E + e] = rows[q * M + lane + 64 * e];
    F::template nat_to_perm<true>(v, rows, tws, lane);
    float2* u = a.u + (size_t)(a.b0 + fb) * N * N;
#pragma unroll
    for (int h = 0; h < F::GPL; ++h)
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            int q;
            const int k = F::perm_k(lane, h, d, q);
            const int iy = iy0 + wave * LPW + q;
            const int ix = (k < H ? k : k - M) + N / 2;
            if (iy < N && ix >= 0 && ix < N) u[(size_t)iy * N + ix] = v[h * 8 + d];
        }
}

// Scaled DFT of one M-point line held by a wave, as two Bluestein
// convolutions of length M (one per half of the outputs) sharing the forward
// transform.  In: natural layout, v[e] = a[lane + 64 e], the pre-chirped input
// in [0, N) and zero above.  Out: natural layout of the M convolution
// outputs.  hh: the plane's two spectra [2][M], FFT order.  LO: N <= M/2, so
// the upper half of the input is zero and the forward transform skips it.
template <int M, bool LO = false>
__device__ __forceinline__ void bluestein_halves(float2* v, float2* scr, const float2* __restrict__ tw,
                                                 const float2* __restrict__ hh, int lane) {
    using F = WaveFFT<M>;
    constexpr int E = F::E, HE = E / 2;
    static_assert(F::LPW == 1 && E % 2 == 0, "one line per wave");
    F::template nat_to_perm<false, LO>(v, scr, tw, lane);
    float2 out[E];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        float2 b[F::NV];
#pragma unroll
        for (int h = 0; h < F::GPL; ++h)
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                int q;
                const int k = F::perm_k(lane, h, d, q);
                b[h * 8 + d] = cmul(v[h * 8 + d], hh[half * M + k]);
            }
        F::template perm_to_nat<true>(b, scr, tw, lane);
        // outputs t = lane + 64 e < M/2 of this half are outputs half * M/2 + t
#pragma unroll
        for (int e = 0; e < HE; ++e) out[half * HE + e] = b[e];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = out[e];
}

// As bluestein_halves, but each output k' (centred k = k' - M/2) is written to
// dst[k mod M] (FFT order) as soon as its half is done, so no registers hold
// the first half while the second is transformed.
template <int M, bool LO = false>
__device__ __forceinline__ void bluestein_halves_to(float2* v, float2* scr, const float2* __restrict__ tw,
                                                    const float2* __restrict__ hh, float2* dst, int lane) {
    using F = WaveFFT<M>;
    constexpr int E = F::E, HE = E / 2;
    static_assert(F::LPW == 1 && E % 2 == 0, "one line per wave");
    F::template nat_to_perm<false, LO>(v, scr, tw, lane);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        float2 b[F::NV];
#pragma unroll
        for (int h = 0; h < F::GPL; ++h)
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                int q;
                const int k = F::perm_k(lane, h, d, q);
                b[h * 8 + d] = cmul(v[h * 8 + d], hh[half * M + k]);
            }
        F::template perm_to_nat<true>(b, scr, tw, lane);
#pragma unroll
        for (int e = 0; e < HE; ++e) dst[(half * (M / 2) + lane + 64 * e + M / 2) & (M - 1)] = b[e];
    }
}

// Row pass: 8 rows per block (8 adjacent columns per store of the transposed
// output); 52 KB of LDS per block at M = 512 and at most 80 VGPRs, so three
// blocks share a CU.
constexpr int kChirpWaves = 8;
// Column passes: one Bluestein line per wave, no block-level exchange, four
// waves per block (35 KB of LDS at M = 512 for k_chirp_cols, so four blocks
// share a CU).
constexpr int kChirpColWaves = 4;

// LO (N <= M/2): the input rows fill at most the lower half of the line.
template <int M, bool LO>
__global__ __launch_bounds__(kChirpWaves * 64) __attribute__((amdgpu_waves_per_eu(M >= 1024 ? 1 : 6, 8))) void k_chirp_rows(ChirpArgs a) {
    using F = WaveFFT<M>;
    constexpr int E = F::E;
    constexpr int SCRP = F::SCR;
    constexpr int MP = M + 2;                // staging row of the transposed store (8 rows
                                             // of one column on distinct bank pairs)
    static_assert(MP <= SCRP, "staging must fit the scratch");
    // [kChirpWaves][SCRP] FFT scratch (later [kChirpWaves][MP] staging), twiddles
    // [M], the plane's chirp spectra [2][M] and chirp [M]
    extern __shared__ float2 sm[];
    float2* tws = sm + kChirpWaves * SCRP;
    float2* hh = tws + M;
    float2* cz = hh + 2 * M;                 // c[m] at m + M/2
    // neighbouring row blocks (which share the cache lines of the transposed
    // store) run on the same XCD
    const int item = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int p = item / gridDim.x;
    const int b = a.g.b0 + p / a.g.nzc, iz = a.g.z0 + p % a.g.nzc;
    for (int i = threadIdx.x; i < M; i += kChirpWaves * 64) {
        tws[i] = a.tw_m[i];
        cz[i] = a.chirp[(size_t)iz * M + i];
    }
    for (int i = threadIdx.x; i < 2 * M; i += kChirpWaves * 64) hh[i] = a.hhat[(size_t)iz * 2 * M + i];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int N = a.N;
    const int iy0 = (item % gridDim.x) * kChirpWaves;
    const int iy = iy0 + wave;
    const int D = M / 2 - N / 2;                           // c of n - N/2 at n + D
    const float2* urow = a.u + ((size_t)b * N + (iy < N ? iy : 0)) * N;
    float2 v[F::NV];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int n = lane + 64 * e;
        v[e] = make_float2(0.f, 0.f);
        if ((!LO || 2 * e < E) && iy < N && n < N) v[e] = cmul(urow[n], cz[n + D]);
    }
    float2* scr = sm + wave * SCRP;
    bluestein_halves<M, LO>(v, scr, tws, hh, lane);
    // outputs k' = lane + 64 e < M: S[k] with k = k' - M/2, stored at kx = k mod M
    // in the block's staging rows (they overlap other waves' scratch: barrier)
    __syncthreads();
    float2* stage = sm + wave * MP;
    const float2 cy = cz[(iy < N ? iy : 0) + D];             // input chirp of the y pass
#pragma unroll
    for (int e = 0; e < M / 64; ++e) {
        const int kp = lane + 64 * e;
        const int k = kp - M / 2;
        stage[(k + M) & (M - 1)] = cmul(cmul(v[e], cz[kp]), cy);
    }
    __syncthreads();
    float2* S1 = a.S1t + (size_t)p * M * N;
    for (int i = threadIdx.x; i < M * kChirpWaves; i += kChirpWaves * 64) {
        const int kx = i / kChirpWaves, j = i % kChirpWaves;
        if (iy0 + j < N) S1[(size_t)kx * N + iy0 + j] = sm[j * MP + kx];
    }
}

// HALF (N <= M/2 and ny <= M/2): the Bluestein input lines fill at most the
// lower half (the forward transform skips the rest), and the window rows lie
// within |m| < M/4, so the output slots e with M/4 <= 64 e < 3M/4 are never
// stored and the final inverse transform does not form them.
template <int M, bool HALF>
__global__ __launch_bounds__(kChirpColWaves * 64) void k_chirp_cols(ChirpArgs a) {
    using F = WaveFFT<M>;
    constexpr int H = M / 2, E = F::E;
    static_assert(F::LPW == 1, "scaled RSD needs M >= 512 per wave line");
    constexpr int SCRP = F::SCR + 1;
    // [kChirpColWaves][SCRP] FFT scratch, [kChirpColWaves][M] scaled spectrum
    // lines, twiddles [M]
    extern __shared__ float2 sm[];
    float2* lines = sm + kChirpColWaves * SCRP;
    float2* tws_m = lines + kChirpColWaves * M;
    const int p = blockIdx.y;
    const int iz = a.g.z0 + p % a.g.nzc;
    const float2* hh = a.hhat + (size_t)iz * 2 * M;     // read through the caches (LDS is the occupancy limit)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kx = blockIdx.x * kChirpColWaves + wave;
    const int N = a.N;
    float2* scr = sm + wave * SCRP;
    float2* line = lines + wave * M;
    // kernel spectrum line Ghat'[kx][ky] (permuted), from the quadrant rows;
    // requested before the twiddle table is staged so both reads overlap
    const float2* Bt = a.Bt + (size_t)p * (H + 1) * a.BS;
    float2 g[F::NV];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int n = lane + 64 * e;
        g[e] = kx <= H ? load_last(&Bt[(size_t)kx * a.BS + (n <= H ? n : M - n)]) : make_float2(0.f, 0.f);
    }
    for (int i = threadIdx.x; i < M; i += kChirpColWaves * 64) tws_m[i] = a.tw_m[i];
    __syncthreads();
    if (kx > H) return;                      // wave-uniform; no block barriers below
    F::template nat_to_perm<false>(g, scr, tws_m, lane);
    // fold the output chirp c[ky] into the kernel line
    const float2* cz = a.chirp + (size_t)iz * M;
#pragma unroll
    for (int h = 0; h < F::GPL; ++h)
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            int q;
            const int k = F::perm_k(lane, h, d, q);
            g[h * 8 + d] = cmul(g[h * 8 + d], cz[(k + M / 2) & (M - 1)]);
        }
    const float2* S1 = a.S1t + (size_t)p * M * N;
    float2* Yp = a.Yt + (size_t)p * M * a.ny;
    const int half = a.ny / 2;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int s = side ? ((M - kx) & (M - 1)) : kx;
        if (side && s == kx) break;
        float2 v[F::NV];
        const float2* srow = S1 + (size_t)s * N + lane;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            v[e] = make_float2(0.f, 0.f);
            if ((!HALF || 2 * e < E) && lane + 64 * e < N) v[e] = load_last(srow + 64 * e);
        }
        // scaled spectrum column S[s][ky] / c[ky], in FFT order in LDS
        bluestein_halves_to<M, HALF>(v, scr, tws_m, hh, line, lane);
        NURSD_WAVE_SYNC();
        float2 x[F::NV];
#pragma unroll
        for (int h = 0; h < F::GPL; ++h)
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                int q;
                const int k = F::perm_k(lane, h, d, q);
                x[h * 8 + d] = cmul(line[k], g[h * 8 + d]);
            }
        NURSD_WAVE_SYNC();
        F::template perm_to_nat<true>(x, scr, tws_m, lane);
        // slot e at a constant offset from one row base (64 e, or 64 e - M
        // past the centre)
        float2* row = Yp + (size_t)s * a.ny + half + lane;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (HALF && 64 * e >= M / 4 && 64 * e < 3 * M / 4) continue;
            const int off = 64 * e < H ? 64 * e : 64 * e - M;
            const int iyo = lane + off + half;
            if (iyo >= 0 && iyo < a.ny) row[off] = x[e];
        }
    }
}

// Voxel-list output on the scaled planes (eq. NURSD2_SRSD): as k_chirp_cols
// up to the product S[s][ky] Ghat'[kx][ky]; then the type-2 steps of the
// NUFFT section along y: deconvolve by the kernel's Fourier coefficients in
// x and y, zero-pad to the 2M-point oversampled line, inverse FFT
// -> T2[p][s][jy].  The Bluestein lines (length M) run in the first M slots of
// the scratch of the 2M-point oversampled line.
// LO (N <= M/2): the Bluestein input lines fill at most the lower half.
template <int M, bool LO>
__global__ __launch_bounds__(kChirpColWaves * 64) void k_chirp_type2_cols(ChirpArgs a) {
    using F = WaveFFT<M>;
    using B = WaveFFT<2 * M>;
    constexpr int H = M / 2, LB = 2 * M, EB = B::E, E = F::E, MF = 2 * M;
    static_assert(F::LPW == 1, "scaled RSD needs M >= 512 per wave line");
    constexpr int SCRP = B::SCR + 1;
    static_assert(SCRP >= MF, "oversampled line must fit the scratch");
    extern __shared__ float2 sm[];           // [kChirpColWaves][SCRP], twiddles LB, twiddles M
    float2* tws_lb = sm + kChirpColWaves * SCRP;
    float2* tws_m = tws_lb + LB;
    for (int i = threadIdx.x; i < LB; i += kChirpColWaves * 64) tws_lb[i] = a.tw_lb[i];
    for (int i = threadIdx.x; i < M; i += kChirpColWaves * 64) tws_m[i] = a.tw_m[i];
    __syncthreads();
    const int p = blockIdx.y;
    const int iz = a.g.z0 + p % a.g.nzc;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kx = blockIdx.x * kChirpColWaves + wave;
    if (kx > H) return;                      // wave-uniform; no block barriers below
    const int N = a.N;
    const float2* hh = a.hhat + (size_t)iz * 2 * M;
    float2* scr = sm + wave * SCRP;
    const float2* Bt = a.Bt + (size_t)p * (H + 1) * a.BS;
    float2 g[F::NV];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int n = lane + 64 * e;
        g[e] = load_last(&Bt[(size_t)kx * a.BS + (n <= H ? n : M - n)]);
    }
    F::template nat_to_perm<false>(g, scr, tws_m, lane);
    // fold the output chirp c[ky] into the kernel line
    const float2* cz = a.chirp + (size_t)iz * M;
#pragma unroll
    for (int h = 0; h < F::GPL; ++h)
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            int q;
            const int k = F::perm_k(lane, h, d, q);
            g[h * 8 + d] = cmul(g[h * 8 + d], cz[(k + M / 2) & (M - 1)]);
        }
    const float2* S1 = a.S1t + (size_t)p * M * N;
    float2* T2 = a.T2 + (size_t)p * M * MF;
    const int lo = a.row_lo[iz], hi = a.row_hi[iz];     // fine rows the row pass reads
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int s = side ? ((M - kx) & (M - 1)) : kx;
        if (side && s == kx) break;
        float2 v[B::NV];
        const float2* srow = S1 + (size_t)s * N + lane;
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            v[e] = make_float2(0.f, 0.f);
            if ((!LO || 2 * e < E) && lane + 64 * e < N) v[e] = load_last(srow + 64 * e);
        }
        bluestein_halves<M, LO>(v, scr, tws_m, hh, lane);
        // scaled spectrum column S[s][ky] / c[ky] (natural), staged to LDS in FFT order
        NURSD_WAVE_SYNC();
#pragma unroll
        for (int e = 0; e < M / 64; ++e) {
            const int k = lane + 64 * e - M / 2;
            scr[(k + M) & (M - 1)] = v[e];
        }
        NURSD_WAVE_SYNC();
        const float dxs = a.dec[s];
        float2 x[F::NV];
#pragma unroll
        for (int h = 0; h < F::GPL; ++h)
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                int q;
                const int k = F::perm_k(lane, h, d, q);
                x[h * 8 + d] = cscale(cmul(scr[k], g[h * 8 + d]), dxs * a.dec[k]);
            }
        // zero-padded natural oversampled line
        NURSD_WAVE_SYNC();
        for (int i = lane; i < MF; i += 64) scr[i] = make_float2(0.f, 0.f);
        NURSD_WAVE_SYNC();
#pragma unroll
        for (int h = 0; h < F::GPL; ++h)
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                int q;
                const int k = F::perm_k(lane, h, d, q);        // ky mod M
                scr[k < H ? k : k + (MF - M)] = x[h * 8 + d];  // ky mod MF
            }
        NURSD_WAVE_SYNC();
#pragma unroll
        for (int e = 0; e < EB; ++e) v[e] = scr[lane + 64 * e];
        B::template nat_to_perm<true>(v, scr, tws_lb, lane);
        float2* trow = T2 + (size_t)s * MF;
#pragma unroll
        for (int h = 0; h < B::GPL; ++h)
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                int q;
                const int jy = B::perm_k(lane, h, d, q);
                if (type2_row_stored(jy, lo, hi, MF)) trow[jy] = v[h * 8 + d];
            }
    }
}

template <typename Args>
static hipError_t launch_k(void (*k)(Args), dim3 grid, int threads, size_t sh, hipStream_t s, const Args& a) {
    if (sh > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, grid, dim3(threads), sh, s, a);
    return hipGetLastError();
}

#define NURSD_SWITCH_M2(M_, CALL)                          \
    switch (M_) {                                          \
        case 64: { constexpr int MM = 64; CALL; }          \
        case 128: { constexpr int MM = 128; CALL; }        \
        case 256: { constexpr int MM = 256; CALL; }        \
        case 512: { constexpr int MM = 512; CALL; }        \
        case 1024: { constexpr int MM = 1024; CALL; }      \
        default: return hipErrorInvalidValue;              \
    }

hipError_t launch_relay_grid(const RelayGridArgs& a, hipStream_t s) {
    NURSD_SWITCH_M2(a.M, {
        using F = WaveFFT<MM>;
        constexpr int LB = kGridWaves * F::LPW;
        hipError_t e = launch_k(k_relay_grid_rows<MM>, dim3((MM + LB - 1) / LB, a.nb), kGridWaves * 64,
                                (size_t)(kGridWaves * F::SCR + MM) * sizeof(float2), s, a);
        if (e != hipSuccess) return e;
        constexpr int SCRP = (F::SCR > F::LPW * MM ? F::SCR : F::LPW * MM) + 1;
        return launch_k(k_relay_grid_cols<MM>, dim3((a.N + LB - 1) / LB, a.nb), kGridWaves * 64,
                        (size_t)(kGridWaves * SCRP + MM) * sizeof(float2), s, a);
    })
}

template <int M>
static hipError_t chirp_rows_m(const ChirpArgs& a, hipStream_t s) {
    using F = WaveFFT<M>;
    const dim3 grid((a.N + kChirpWaves - 1) / kChirpWaves, a.g.nb * a.g.nzc);
    const size_t sh = (size_t)(kChirpWaves * F::SCR + 4 * M) * sizeof(float2);
    if (2 * a.N <= M) return launch_k(k_chirp_rows<M, true>, grid, kChirpWaves * 64, sh, s, a);
    return launch_k(k_chirp_rows<M, false>, grid, kChirpWaves * 64, sh, s, a);
}

template <int M>
static hipError_t chirp_cols_m(const ChirpArgs& a, hipStream_t s) {
    using F = WaveFFT<M>;
    const dim3 grid((M / 2 + 1 + kChirpColWaves - 1) / kChirpColWaves, a.g.nb * a.g.nzc);
    const size_t sh = (size_t)(kChirpColWaves * (F::SCR + 1 + M) + M) * sizeof(float2);
    if (2 * a.N <= M && 2 * a.ny <= M) return launch_k(k_chirp_cols<M, true>, grid, kChirpColWaves * 64, sh, s, a);
    return launch_k(k_chirp_cols<M, false>, grid, kChirpColWaves * 64, sh, s, a);
}

template <int M>
static hipError_t chirp_type2_cols_m(const ChirpArgs& a, hipStream_t s) {
    using B = WaveFFT<2 * M>;
    const dim3 grid((M / 2 + 1 + kChirpColWaves - 1) / kChirpColWaves, a.g.nb * a.g.nzc);
    const size_t sh = (size_t)(kChirpColWaves * (B::SCR + 1) + 2 * M + M) * sizeof(float2);
    if (2 * a.N <= M) return launch_k(k_chirp_type2_cols<M, true>, grid, kChirpColWaves * 64, sh, s, a);
    return launch_k(k_chirp_type2_cols<M, false>, grid, kChirpColWaves * 64, sh, s, a);
}

hipError_t launch_chirp_rows(const ChirpArgs& a, hipStream_t s) {
    switch (a.M) {
        case 512: return chirp_rows_m<512>(a, s);
        case 1024: return chirp_rows_m<1024>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_chirp_cols(const ChirpArgs& a, hipStream_t s) {
    switch (a.M) {
        case 512: return chirp_cols_m<512>(a, s);
        case 1024: return chirp_cols_m<1024>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_chirp_type2_cols(const ChirpArgs& a, hipStream_t s) {
    switch (a.M) {
        case 512: return chirp_type2_cols_m<512>(a, s);
        case 1024: return chirp_type2_cols_m<1024>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace nursd
