// Steps 4-7: per-depth RSD propagation (eq. Discrete_RSD_Conv / eq. NURSD1)
// and volume formation (eq. PF_RSD_Defn).
//
// For every (frequency b, plane z) of a chunk the three passes compute
//   F_{b,z}[m'] = M^-2 sum_k U_b[k] Ghat_{b,z}[k] e^{+2 pi j k.m'/M}
// on the output window, with Ghat the DFT over I_M^2 of the sampled kernel
// G(m dx, n dy, z) = e^{+j 2 pi f r / c} / r.  Ghat is generated on the fly
// and never stored whole.  G is even in m and in n, and the sampled set I_M
// is closed under m -> -m (mod M), so Ghat is a cosine transform of the
// quadrant [0, M/2]^2:
//   P1 (k_kernel_rows): generate the quadrant rows (FP64 phase argument,
//       reduced to a fractional cycle before the FP32 sin/cos) and transform
//       each row along x as an even-extended M-point FFT; keep kx in [0, M/2].
//   P2 (k_propagate_cols): finish Ghat along y for a block of kx, multiply by
//       the spectrum rows U_b[+kx] and U_b[-kx] (Ghat is even in kx), inverse
//       FFT along y and keep the ny output rows of the window.
//   P3 (k_propagate_rows): inverse FFT along x, keep the nx window columns,
//       multiply by the illumination phase e^{+j 2 pi f |x_v - x_p| / c}
//       (FP64 argument) and accumulate over the chunk's frequencies in
//       registers before one read-modify-write of the volume.
#include "kernels.hpp"
#include "persistent.hpp"
#include "wavefft.hpp"

namespace nursd {


// e^{+j 2 pi (r f / c)} / r for r = sqrt(r2); the cycle count r f / c is
// formed in FP64 and reduced to [-1/2, 1/2] before the FP32 sin/cos.
__device__ __forceinline__ float2 rsd_kernel(double r2, double f_over_c) {
    float ir;
    const double r = sqrt_f64(r2, &ir);
    const double cyc = r * f_over_c;
    const float fr = (float)(cyc - rint(cyc));
    float s, c;
    sincos_cycles(fr, &s, &c);
    return make_float2(c * ir, s * ir);
}

// e^{+j 2 pi (r f / c)}: the 3D-RSD kernel (no amplitude), finite at r = 0.
__device__ __forceinline__ float2 rsd_kernel_plain(double r2, double f_over_c) {
    float ir;
    const double r = r2 > 0.0 ? sqrt_f64(r2, &ir) : 0.0;
    const double cyc = r * f_over_c;
    const float fr = (float)(cyc - rint(cyc));
    float s, c;
    sincos_cycles(fr, &s, &c);
    return make_float2(c, s);
}

// e^{+j 2 pi d f / c} for a precomputed distance d.
__device__ __forceinline__ float2 phase_of(double d, double f_over_c) {
    const double cyc = d * f_over_c;
    const float fr = (float)(cyc - rint(cyc));
    float s, c;
    sincos_cycles(fr, &s, &c);
    return make_float2(c, s);
}

__device__ __forceinline__ double dist3(double x, double y, double z) {
    const double d2 = x * x + y * y + z * z;
    float inv;
    return sqrt_f64(d2, &inv);
}

__device__ __forceinline__ void plane_of(const ChunkGeom& g, int p, int& b, int& iz) {
    b = g.b0 + p / g.nzc;
    iz = g.z0 + p % g.nzc;
}

// P1: one wavefront per kernel row my (LPW rows per wave for M < 512).
// Waves per block (compile-time knob; 8 measured fastest, 16 and 4 slower).
#ifndef NURSD_P1_WAVES
#define NURSD_P1_WAVES 8
#endif
constexpr int kP1Waves = NURSD_P1_WAVES;

// Pitch of a wave's scratch row (float2): the FFT scratch plus 2, so that at
// M = 512 the transposed read of the block's output (its 8 rows of one
// column, then of the next) touches distinct LDS bank pairs.
template <int M>
constexpr int p1_scrp() { return WaveFFT<M>::SCR + 2; }

template <int M, int NW = kP1Waves>
__device__ __forceinline__ void kernel_rows_body(const P1Args& a, int bx, int by) {
    using F = WaveFFT<M>;
    constexpr int H = M / 2, E = F::E, LPW = F::LPW, SCRP = p1_scrp<M>();
    extern __shared__ float2 sm[];      // [NW][SCRP], twiddles [TWN], Nyquist samples [LB]
    float2* tws = sm + NW * SCRP;
    for (int i = threadIdx.x; i < F::TWN; i += NW * 64) tws[i] = a.tw[i];
    const int p = by;
    int b, iz;
    plane_of(a.g, p, b, iz);
    const double foc = a.g.f[b] / kC;
    const double z = a.g.z[iz];
    const double px = a.g.pitch_x ? a.g.pitch_x[iz] : a.g.dx;
    const double py = a.g.pitch_y ? a.g.pitch_y[iz] : a.g.dy;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    constexpr int LB = NW * LPW;
    const int my0 = bx * LB;
    // For M >= 128 the sample n = M/2 of a row sits alone in slot E/2 of lane
    // 0; the block computes those LB samples once, one per thread, instead of
    // every wave spending a whole slot on one lane.
    constexpr bool NYQ_LDS = E >= 2;
    float2* nyq = tws + F::TWN;
    if (NYQ_LDS && tid < LB) {
        const int my = my0 + tid;
        const double ry = (my <= H ? my : 0) * py, rx = H * px;
        nyq[tid] = a.plain ? rsd_kernel_plain(fma(rx, rx, fma(ry, ry, z * z)), foc)
                           : rsd_kernel(fma(rx, rx, fma(ry, ry, z * z)), foc);
    }
    __syncthreads();
    // Waves whose rows all lie past M/2 (the tail of the last block) skip
    // the work but still meet the block barriers.
    if (my0 + wave * LPW <= H) {
        float2 v[F::NV];
#pragma unroll
        for (int q = 0; q < LPW; ++q) {
            const int my = my0 + wave * LPW + q;
            const double ry = (my <= H ? my : 0) * py;
            const double ryz = fma(ry, ry, z * z);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int n = lane + 64 * e;
                v[q * E + e] = make_float2(0.f, 0.f);
                if (NYQ_LDS && 64 * e == H) {
                    if (lane == 0 && my <= H) v[q * E + e] = nyq[wave * LPW + q];
                } else if (my <= H && n <= H) {
                    const double rx = n * px;
                    v[q * E + e] = a.plain ? rsd_kernel_plain(fma(rx, rx, ryz), foc) : rsd_kernel(fma(rx, rx, ryz), foc);
                }
            }
            // even extension: x[n] = x[M - n] for n > M/2, taken from the lane
            // that computed M - n (same wave)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (64 * e + 63 <= H) continue;             // no slot of this e exceeds H
                const int n = lane + 64 * e;
                const float2 src = v[q * E + (E - 1 - e >= 0 ? E - 1 - e : 0)];
                float2 t;
                t.x = __shfl(src.x, (64 - lane) & 63);
                t.y = __shfl(src.y, (64 - lane) & 63);
                if (n > H) v[q * E + e] = (lane == 0) ? v[q * E + (E - e < E ? E - e : 0)] : t;
            }
        }
        float2* scr = sm + wave * SCRP;
        F::template nat_to_perm<false>(v, scr, tws, lane);
#pragma unroll
        for (int h = 0; h < F::GPL; ++h)
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                int q;
                const int k = F::perm_k(lane, h, d, q);
                if (k <= H) scr[q * (H + 1) + k] = v[h * 8 + d];
            }
    }
    __syncthreads();
    float2* Bt = a.Bt + (size_t)p * (H + 1) * a.BS;
    for (int i = tid; i < (H + 1) * LB; i += NW * 64) {
        const int kx = i / LB, j = i % LB;
        const int my = my0 + j;
        if (my <= H) Bt[(size_t)kx * a.BS + my] = sm[(j / LPW) * SCRP + (j % LPW) * (H + 1) + kx];
    }
}

// P2: one wavefront per kx line (LPW lines for M < 512): Ghat along y,
// times U[+kx] and U[-kx], inverse along y, window rows -> Yt[p][s][iy].
// Waves per block (compile-time knob): 4 measured fastest (the tail of each
// plane's M/2 + 1 lines wastes less, more blocks fit a CU); 2, 8, 16 slower.
#ifndef NURSD_P2_WAVES
#define NURSD_P2_WAVES 4
#endif
constexpr int kP2Waves = NURSD_P2_WAVES;

// Spectrum product and inverse y transform of a wave's kx lines for one
// target: for s = kx and s = M - kx, Yp[s][iy] = IDFT_y(U[s] * g)[window row
// iy] with g the permuted kernel spectrum line(s).  ny, q: the target's
// window rows and upsampling.
// HALFY (M >= 256, ny q <= M/2): window rows lie within |m| < M/4, so the
// slots e with M/4 <= 64 e < 3M/4 are never stored and the last radix stage
// of the inverse transform only forms the outputs that are.
template <int M, bool HALFY = false>
__device__ __forceinline__ void cols_apply(const float2* g, const float2* __restrict__ Ub, float2* Yp, int ny, int qf,
                                           int kx0, float2* scr, const float2* tws, int lane) {
    using F = WaveFFT<M>;
    constexpr int H = M / 2, E = F::E, LPW = F::LPW;
    static_assert(!HALFY || M >= 256, "row pruning needs quarter periods of whole 64-row slots");
    const int half = ny / 2;
    float2 v[F::NV];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
#pragma unroll
        for (int h = 0; h < F::GPL; ++h)
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                int q;
                const int k = F::perm_k(lane, h, d, q);
                const int kx = kx0 + q;
                const int s = side ? ((M - kx) & (M - 1)) : kx;
                v[h * 8 + d] = kx <= H ? cmul(Ub[(size_t)s * M + k], g[h * 8 + d]) : make_float2(0.f, 0.f);
            }
        F::template perm_to_nat<true>(v, scr, tws, lane);
#pragma unroll
        for (int q = 0; q < LPW; ++q) {
            const int kx = kx0 + q;
            const int s = side ? ((M - kx) & (M - 1)) : kx;
            if (kx > H || (side && s == kx)) continue;
            if (qf == 1) {
                // One row base per line; slot e sits at offset 64 e, or 64 e - M
                // past the centre, which is a constant when M/2 is a multiple of
                // 64, so the stores take immediate offsets.
                float2* row = Yp + (size_t)s * ny + half + lane;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if (HALFY && 64 * e >= M / 4 && 64 * e < 3 * M / 4) continue;
                    const bool lower = H % 64 == 0 ? 64 * e < H : lane + 64 * e < H;
                    const int off = lower ? 64 * e : 64 * e - M;
                    const int iy = lane + off + half;
                    if (iy >= 0 && iy < ny) row[off] = v[q * E + e];
                }
            } else {
                // upsampled frame: window row iy is grid row iy q - (ny q)/2
                const int hq = (ny * qf) / 2;
                float2* row = Yp + (size_t)s * ny;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if (HALFY && 64 * e >= M / 4 && 64 * e < 3 * M / 4) continue;
                    const int n = lane + 64 * e;
                    const int t = (n < H ? n : n - M) + hq;
                    if (t >= 0 && t % qf == 0 && t / qf < ny) row[t / qf] = v[q * E + e];
                }
            }
        }
    }
}

// The kernel quadrant line(s) of the wave's kx lines (even extension along
// y), requested before the block stages the twiddle table so that both
// global reads are in flight across the block barrier.
template <int M>
__device__ __forceinline__ void load_kernel_lines(float2* v, const float2* __restrict__ Bt, int BS, int kx0,
                                                  int lane) {
    using F = WaveFFT<M>;
    constexpr int H = M / 2, E = F::E, LPW = F::LPW;
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
        const int kx = kx0 + q;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int n = lane + 64 * e;
            const int dd = n <= H ? n : M - n;
            v[q * E + e] = kx <= H ? Bt[(size_t)kx * BS + dd] : make_float2(0.f, 0.f);
        }
    }
}

template <int M, int NW = kP2Waves, bool HALFY = false>
__device__ __forceinline__ void propagate_cols_body(const P2Args& a, int bx, int by) {
    using F = WaveFFT<M>;
    constexpr int H = M / 2;
    extern __shared__ float2 sm[];      // [NW][SCR], then twiddles [M]
    float2* tws = sm + NW * F::SCR;
    const int p = by;
    int b, iz;
    plane_of(a.g, p, b, iz);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int kx0 = (bx * NW + wave) * F::LPW;
    float2* scr = sm + wave * F::SCR;
    const int kp = a.kidx ? a.kidx[b * a.kz + iz] : p;
    float2 g[F::NV];
    load_kernel_lines<M>(g, a.Bt + (size_t)kp * (H + 1) * a.BS, a.BS, kx0, lane);
    for (int i = threadIdx.x; i < M; i += NW * 64) tws[i] = a.tw[i];
    __syncthreads();
    if (kx0 > H) return;                // wave-uniform; no block barriers below
    F::template nat_to_perm<false>(g, scr, tws, lane);
    cols_apply<M, HALFY>(g, a.U + (size_t)b * M * M, a.Yt + (size_t)p * M * a.ny, a.ny, a.q, kx0, scr, tws, lane);
}

// Batched mode, one kernel spectrum line for many scenes: block (bx, item)
// transforms the kernel lines of table plane kp[item] once and applies them
// to every user of that plane (a scene's spectrum at the user's frequency
// and its output plane).
template <int M, int NW = kP2Waves, bool HALFY = false>
__device__ __forceinline__ void propagate_cols_multi_body(const P2MArgs& a, int bx, int item) {
    using F = WaveFFT<M>;
    constexpr int H = M / 2;
    extern __shared__ float2 sm[];      // [NW][SCR], then twiddles [M]
    float2* tws = sm + NW * F::SCR;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int kx0 = (bx * NW + wave) * F::LPW;
    float2* scr = sm + wave * F::SCR;
    float2 g[F::NV];
    load_kernel_lines<M>(g, a.Bt + (size_t)a.kp[item] * (H + 1) * a.BS, a.BS, kx0, lane);
    for (int i = threadIdx.x; i < M; i += NW * 64) tws[i] = a.tw[i];
    __syncthreads();
    if (kx0 > H) return;                // wave-uniform; no block barriers below
    F::template nat_to_perm<false>(g, scr, tws, lane);
    const int u1 = a.user_ptr[item + 1];
    for (int u = a.user_ptr[item]; u < u1; ++u) {
        const P2MUser us = a.users[u];
        cols_apply<M, HALFY>(g, us.U, us.Yt, us.ny, us.q, kx0, scr, tws, lane);
    }
}

// P3: LPW output rows per wavefront, RB = waves * LPW rows per block; loops
// over the chunk's frequencies with per-voxel accumulators in registers.
// The block's column tile of the next frequency is loaded into registers
// while the current one is transformed, so that HBM reads overlap the FFT.
// The chunk's frequencies are evenly spaced (the host splits uneven bin
// lists into single-frequency chunks), so the illumination phase of each
// voxel is advanced by a step factor e^{+j 2 pi df d / c} (both factors from
// FP64 arguments) instead of being evaluated per frequency.
#ifndef NURSD_P3_WAVES
#define NURSD_P3_WAVES 16
#endif
// The full-window variant keeps twice the per-voxel state and runs 8 waves
// per block so that it fits the register file without spilling.
template <int M, bool HALF>
constexpr int p3_waves() { return (M >= 1024 || !HALF) ? 8 : NURSD_P3_WAVES; }

// With nx <= M/2 (zero padding >= 2) only permuted slots d in {0, 1, 6, 7}
// of each 8-point group can fall inside the window (|m'| < M/4); HALF keeps
// per-voxel state for those four slots only.
// The persistent (grouped) launches run 4 or 8 waves per block: with the
// work-queue loop around the body, 16 waves (128 VGPRs each) spill.

// Row pitch of the last pass's tile (float2): a wave's FFT scratch or its
// LPW output rows, plus NURSD_P3_PAD.
#ifndef NURSD_P3_PAD
#define NURSD_P3_PAD 1
#endif
template <int M>
constexpr int p3_scrp() {
    using F = WaveFFT<M>;
    return (F::SCR > F::LPW * M ? F::SCR : F::LPW * M) + NURSD_P3_PAD;
}

template <int M, bool HALF, int NW = p3_waves<M, HALF>()>
__device__ __forceinline__ void propagate_rows_body(const P3Args& a, int bx, int by) {
    using F = WaveFFT<M>;
    constexpr int H = M / 2, E = F::E, LPW = F::LPW;
    constexpr int SCRP = p3_scrp<M>();
    constexpr int RB = NW * LPW;
    constexpr int NPRE = M * RB / (NW * 64);     // tile values per thread
    static_assert(M * RB % (NW * 64) == 0, "tile must divide over the block");
    extern __shared__ float2 sm[];      // two tiles [2][NW][SCRP], then twiddles [M]
    float2* tws = sm + 2 * NW * SCRP;
    // (staged before the tile request: loads complete in order, so waiting
    // for the table after it would wait for the tile too)
    for (int i = threadIdx.x; i < M; i += NW * 64) tws[i] = a.tw[i];
    const int zl = by;
    const int iz = a.g.z0 + zl;
    const int iy0 = bx * RB;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int nx = a.nx, ny = a.ny;
    const double z = a.g.z[iz];
    const double px = a.g.pitch_x ? a.g.pitch_x[iz] : a.g.dx;
    const double py = a.g.pitch_y ? a.g.pitch_y[iz] : a.g.dy;
    const size_t plane_off = (size_t)iz * ny * nx;
    const int b_end = a.g.b0 + a.g.nb;
    // This thread's share of the block's column tile: entry i = tid + r * NW * 64
    // holds column s = i / RB of output row iy0 + i % RB.  Since NW * 64 is a
    // multiple of RB, the row is tid % RB for every r and the column steps by
    // 64 / LPW.  Rows past ny (ragged last block) load row ny - 1 instead:
    // their transforms are never stored, and the loads need no branch.  The
    // first tile is requested before the per-voxel set-up below, which then
    // overlaps its latency.
    float2 pre[NPRE];
    const float2* Yb = a.Yt + (size_t)zl * M * ny;
    const size_t fstride = (size_t)a.g.nzc * M * ny;  // next frequency, same plane
    static_assert((NW * 64) % RB == 0, "tile rows repeat with period RB");
    const unsigned toff = (unsigned)((tid / RB) * ny + min(iy0 + tid % RB, ny - 1));
    const unsigned tstep = (unsigned)((64 / LPW) * ny);
#pragma unroll
    for (int r = 0; r < NPRE; ++r) pre[r] = Yb[toff + r * tstep];
    constexpr int SPG = HALF ? 4 : 8;                   // kept slots per 8-point group
    constexpr int NS = F::GPL * SPG;
    const double f0c = a.g.f[a.g.b0] / kC, dfc = a.g.df / kC;   // cycles per metre
    float2 acc[NS], ph[NS], st[NS];
    int off[NS];                        // output offset within the plane, -1 outside the window
#pragma unroll
    for (int h = 0; h < F::GPL; ++h)
#pragma unroll
        for (int j = 0; j < SPG; ++j) {
            const int d = HALF ? (j < 2 ? j : j + 4) : j;
            const int sl = h * SPG + j;
            int q;
            const int k = F::perm_k(lane, h, d, q);
            const int iy = iy0 + wave * LPW + q;
            // grid column m of the frame is window column (m + (nx q)/2) / q
            // when that divides (q = 1: every column)
            const int m = k < H ? k : k - M;
            const int t = m + (nx * a.q) / 2;
            const int ix = (t >= 0 && t % a.q == 0) ? t / a.q : -1;
            off[sl] = (iy < ny && ix >= 0 && ix < nx) ? iy * nx + ix : -1;
            acc[sl] = make_float2(0.f, 0.f);
            ph[sl] = make_float2(1.f, 0.f);
            st[sl] = make_float2(1.f, 0.f);
            if (off[sl] >= 0) {
                const double x = a.xc + m * px;
                const double y = a.yc + (iy * a.q - (ny * a.q) / 2) * py;
                const double dd = dist3(x - a.xp0, y - a.xp1, z - a.xp2);
                ph[sl] = phase_of(dd, f0c);
                st[sl] = phase_of(dd, dfc);
                if (!a.first) {
                    if (a.coherent) acc[sl] = a.V[plane_off + off[sl]];
                    else acc[sl].x = a.I[plane_off + off[sl]];
                }
            }
        }
    // Two tiles alternate: while the waves transform their rows of frequency b
    // (each wave uses its own row of the tile as FFT scratch), frequency b+1 is
    // stored into the other tile and b+2 is loaded, with one barrier per step.
    auto store_tile = [&](float2* tile) {
#pragma unroll
        for (int r = 0; r < NPRE; ++r) {
            const int i = tid + r * NW * 64;
            const int s = i / RB, j = i % RB;
            tile[(j / LPW) * SCRP + (j % LPW) * M + s] = pre[r];
        }
    };
    auto load_tile = [&]() {
        Yb += fstride;
#pragma unroll
        for (int r = 0; r < NPRE; ++r) pre[r] = Yb[toff + r * tstep];
    };
    store_tile(sm);
    if (a.g.b0 + 1 < b_end) load_tile();
    for (int b = a.g.b0; b < b_end; ++b) {
        __syncthreads();
        float2* cur = sm + ((b - a.g.b0) & 1) * NW * SCRP;
        float2* rows = cur + wave * SCRP;
        float2 v[F::NV];
#pragma unroll
        for (int q = 0; q < LPW; ++q)
#pragma unroll
            for (int e = 0; e < E; ++e) v[q * E + e] = rows[q * M + lane + 64 * e];
        F::template nat_to_perm<true>(v, rows, tws, lane);
        // The other tile is free since the barrier: the next frequency's tile
        // is stored after this wave's transform (so the waves' LDS writes
        // spread over the others' FFTs) and the one after is requested.
        if (b + 1 < b_end) {
            store_tile(sm + ((b + 1 - a.g.b0) & 1) * NW * SCRP);
            if (b + 2 < b_end) load_tile();
        }
#pragma unroll
        for (int h = 0; h < F::GPL; ++h)
#pragma unroll
            for (int j = 0; j < SPG; ++j) {
                const int d = HALF ? (j < 2 ? j : j + 4) : j;
                const int sl = h * SPG + j;
                const float2 val = v[h * 8 + d];
                if (off[sl] < 0) continue;
                if (a.field) {
                    a.field[(size_t)(b * a.field_nz + iz - a.field_z0) * ny * nx + off[sl]] = cmul(ph[sl], val);
                    ph[sl] = cmul(ph[sl], st[sl]);
                } else if (a.coherent) {
                    acc[sl] = cadd(acc[sl], cmul(ph[sl], val));
                    ph[sl] = cmul(ph[sl], st[sl]);
                } else {
                    acc[sl].x += sqrtf(val.x * val.x + val.y * val.y);
                }
            }
    }
    if (a.field) return;
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
        if (off[sl] < 0) continue;
        const size_t o = plane_off + off[sl];
        if (a.coherent) {
            a.V[o] = acc[sl];
            if (a.last && a.I) a.I[o] = sqrtf(acc[sl].x * acc[sl].x + acc[sl].y * acc[sl].y);
        } else {
            a.I[o] = acc[sl].x;
        }
    }
}

template <int M>
__global__ __launch_bounds__(kP1Waves * 64) void k_kernel_rows(P1Args a) {
    kernel_rows_body<M>(a, blockIdx.x, blockIdx.y);
}
// Grouped (batched) variants take the waves per block as a template
// parameter: the batch's tuner picks one per transform size.
template <int M, int NW>
__global__ __launch_bounds__(NW * 64, (M >= 1024 ? 4 : 8)) void k_kernel_rows_grouped(Group<P1Args> g) {
    persistent_loop(g, [](const P1Args& a, int bx, int by) { kernel_rows_body<M, NW>(a, bx, by); });
}
// The column pass renumbers its workgroups (xcd_contiguous) so that each XCD
// works through a contiguous run of (plane, kx block) work items: the planes
// of one frequency share its spectrum U, which then stays in that XCD's L2.

template <int M, bool HALFY>
__global__ __launch_bounds__(kP2Waves * 64) void k_propagate_cols(P2Args a) {
    const int v = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    propagate_cols_body<M, kP2Waves, HALFY>(a, v % gridDim.x, v / gridDim.x);
}
template <int M, int NW, bool HALFY>
__global__ __launch_bounds__(NW * 64) void k_propagate_cols_grouped(Group<P2Args> g) {
    persistent_loop(g, [](const P2Args& a, int bx, int by) { propagate_cols_body<M, NW, HALFY>(a, bx, by); });
}
template <int M, bool HALFY>
__global__ __launch_bounds__(kP2Waves * 64) void k_propagate_cols_multi(P2MArgs a) {
    const int2 w = a.blk[blockIdx.x];
    propagate_cols_multi_body<M, kP2Waves, HALFY>(a, w.y, w.x);
}
template <int M, bool HALF>
__global__ __launch_bounds__((p3_waves<M, HALF>() * 64)) void k_propagate_rows(P3Args a) {
    const int v = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    propagate_rows_body<M, HALF>(a, v % gridDim.x, v / gridDim.x);
}
template <int M, bool HALF, int NW>
__global__ __launch_bounds__(NW * 64) void k_propagate_rows_grouped(Group<P3Args> g) {
    persistent_loop(g, [](const P3Args& a, int bx, int by) { propagate_rows_body<M, HALF, NW>(a, bx, by); });
}

template <typename Args>
static hipError_t launch_rsd(void (*k)(Args), dim3 grid, int threads, size_t sh, hipStream_t s, const Args& a) {
    if (sh > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, grid, dim3(threads), sh, s, a);
    return hipGetLastError();
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

#define NURSD_SWITCH_M(M_, CALL)                           \
    switch (M_) {                                          \
        case 64: { constexpr int MM = 64; CALL; }          \
        case 128: { constexpr int MM = 128; CALL; }        \
        case 256: { constexpr int MM = 256; CALL; }        \
        case 512: { constexpr int MM = 512; CALL; }        \
        case 1024: { constexpr int MM = 1024; CALL; }      \
        default: return hipErrorInvalidValue;              \
    }

hipError_t launch_kernel_rows(const P1Args& a, hipStream_t s) {
    const int planes = a.g.nb * a.g.nzc;
    NURSD_SWITCH_M(a.M, {
        using F = WaveFFT<MM>;
        constexpr int LB = kP1Waves * F::LPW;
        dim3 grid((MM / 2 + 1 + LB - 1) / LB, planes);
        return launch_rsd(k_kernel_rows<MM>, grid, kP1Waves * 64,
                          (size_t)(kP1Waves * p1_scrp<MM>() + F::TWN + kP1Waves * F::LPW) * sizeof(float2),
                          s, a);
    })
}

hipError_t launch_propagate_cols(const P2Args& a, hipStream_t s) {
    const int planes = a.g.nb * a.g.nzc;
    NURSD_SWITCH_M(a.M, {
        using F = WaveFFT<MM>;
        constexpr int LB = kP2Waves * F::LPW;
        dim3 grid((MM / 2 + 1 + LB - 1) / LB, planes);
        const size_t sh = (size_t)(kP2Waves * F::SCR + MM) * sizeof(float2);
        if (MM >= 256 && 2 * a.ny * a.q <= MM)
            return launch_rsd(k_propagate_cols<MM, (MM >= 256)>, grid, kP2Waves * 64, sh, s, a);
        return launch_rsd(k_propagate_cols<MM, false>, grid, kP2Waves * 64, sh, s, a);
    })
}

hipError_t launch_propagate_cols_multi(const P2MArgs& a, int nblk, bool halfy, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    NURSD_SWITCH_M(a.M, {
        using F = WaveFFT<MM>;
        const size_t sh = (size_t)(kP2Waves * F::SCR + MM) * sizeof(float2);
        if (halfy && MM >= 256)
            return launch_rsd(k_propagate_cols_multi<MM, (MM >= 256)>, dim3(nblk), kP2Waves * 64, sh, s, a);
        return launch_rsd(k_propagate_cols_multi<MM, false>, dim3(nblk), kP2Waves * 64, sh, s, a);
    })
}
int grid_x_propagate_cols_multi(int M) { return grid_x_propagate_cols(M, kP2Waves); }

hipError_t launch_propagate_rows(const P3Args& a, hipStream_t s) {
    if (!a.g.uni) return hipErrorInvalidValue;     // phases advance by a fixed step
    if (a.q < 1) return hipErrorInvalidValue;
    const bool half = 2 * a.nx * a.q <= a.M;
    NURSD_SWITCH_M(a.M, {
        using F = WaveFFT<MM>;
        constexpr int SCRP = p3_scrp<MM>();
        if (half) {
            constexpr int NW = (p3_waves<MM, true>());
            constexpr int RB = NW * F::LPW;
            return launch_rsd((k_propagate_rows<MM, true>), dim3((a.ny + RB - 1) / RB, a.g.nzc), NW * 64,
                              (size_t)(2 * NW * SCRP + MM) * sizeof(float2), s, a);
        }
        constexpr int NW = (p3_waves<MM, false>());
        constexpr int RB = NW * F::LPW;
        return launch_rsd((k_propagate_rows<MM, false>), dim3((a.ny + RB - 1) / RB, a.g.nzc), NW * 64,
                          (size_t)(2 * NW * SCRP + MM) * sizeof(float2), s, a);
    })
}

template <int M, int W>
static hipError_t p1_grouped(const Group<P1Args>& g, hipStream_t s) {
    using F = WaveFFT<M>;
    return launch_grouped(k_kernel_rows_grouped<M, W>, g, W * 64,
                          (size_t)(W * p1_scrp<M>() + F::TWN + W * F::LPW) * sizeof(float2), s);
}
template <int M, int W>
static hipError_t p2_grouped(bool halfy, const Group<P2Args>& g, hipStream_t s) {
    using F = WaveFFT<M>;
    constexpr size_t sh = (size_t)(W * F::SCR + M) * sizeof(float2);
    if (halfy && M >= 256) return launch_grouped(k_propagate_cols_grouped<M, W, (M >= 256)>, g, W * 64, sh, s);
    return launch_grouped(k_propagate_cols_grouped<M, W, false>, g, W * 64, sh, s);
}
template <int M, int W>
static hipError_t p3_grouped(bool half, const Group<P3Args>& g, hipStream_t s) {
    constexpr int SCRP = p3_scrp<M>();
    constexpr size_t sh = (size_t)(2 * W * SCRP + M) * sizeof(float2);
    if (half) return launch_grouped(k_propagate_rows_grouped<M, true, W>, g, W * 64, sh, s);
    return launch_grouped(k_propagate_rows_grouped<M, false, W>, g, W * 64, sh, s);
}
template <int M>
static hipError_t p1_grouped_m(int nw, const Group<P1Args>& g, hipStream_t s) {
    switch (nw) {
        case 4: return p1_grouped<M, 4>(g, s);
        case 8: return p1_grouped<M, 8>(g, s);
        default: return hipErrorInvalidValue;
    }
}
template <int M>
static hipError_t p2_grouped_m(bool halfy, int nw, const Group<P2Args>& g, hipStream_t s) {
    switch (nw) {
        case 2: return p2_grouped<M, 2>(halfy, g, s);
        case 4: return p2_grouped<M, 4>(halfy, g, s);
        case 8: return p2_grouped<M, 8>(halfy, g, s);
        default: return hipErrorInvalidValue;
    }
}
template <int M>
static hipError_t p3_grouped_m(bool half, int nw, const Group<P3Args>& g, hipStream_t s) {
    switch (nw) {
        case 4: return p3_grouped<M, 4>(half, g, s);
        case 8: return p3_grouped<M, 8>(half, g, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_kernel_rows_grouped(int M, int nw, const Group<P1Args>& g, hipStream_t s) {
    NURSD_SWITCH_M(M, return p1_grouped_m<MM>(nw, g, s));
}

hipError_t launch_propagate_cols_grouped(int M, bool halfy, int nw, const Group<P2Args>& g, hipStream_t s) {
    NURSD_SWITCH_M(M, return p2_grouped_m<MM>(halfy, nw, g, s));
}

hipError_t launch_propagate_rows_grouped(int M, bool half, int nw, const Group<P3Args>& g, hipStream_t s) {
    NURSD_SWITCH_M(M, return p3_grouped_m<MM>(half, nw, g, s));
}

// Blocks along x of one (plane or depth) of the three passes at M with nw
// waves per block.
int grid_x_kernel_rows(int M, int nw) {
    const int lpw = M >= 512 ? 1 : 512 / M;
    return (M / 2 + 1 + nw * lpw - 1) / (nw * lpw);
}
int grid_x_propagate_cols(int M, int nw) {
    const int lpw = M >= 512 ? 1 : 512 / M;
    return (M / 2 + 1 + nw * lpw - 1) / (nw * lpw);
}
int rows_per_block_propagate(int M, int nw) {
    const int lpw = M >= 512 ? 1 : 512 / M;
    return nw * lpw;
}

}  // namespace nursd
