// Step 8: adjoint of the coherent uniform-grid operator P -> V and the
// relay-position gradient.
//
// Forward (per frequency b, plane z, window voxel m'):
//   V[z][m'] += Phi_b(m', z) sum_k Us_b[k] Ghat_{b,z}[k] e^{+2 pi j k.m'/M},
//   Us_b = M^-2 NUFFT1(P_b),  Phi_b = e^{+j 2 pi f_b |x_v - x_p| / c}.
// Adjoint, for an upstream gradient gV (dL/dRe V + j dL/dIm V):
//   St_b[k] = sum_z conj(Ghat_{b,z}[k]) sum_{m'} e^{-2 pi j k.m'/M} conj(Phi_b) gV[z][m']
//   grad_P[b][l] = M^-2 sum_k St_b[k] e^{+j k.x~_l}                   (type-2 NUFFT)
//   grad_x[l] = Re sum_b conj(P_bl) M^-2 sum_k St_b[k] (j 2 pi kx / Lx) e^{+j k.x~_l}
// (and likewise y), the derivative of the type-1 sum with respect to x_l.
// Nothing is kept from the forward pass: the kernel spectra are recomputed
// per frequency (k_kernel_rows), which is the per-frequency checkpointing.
//   k_adj_rows:  conj phase times gV on each window row, zero-padded forward
//                FFT along x, transposed store Rt[p][kx][iy].
//   k_adj_cols:  forward FFT along y of Rt rows +kx and -kx, times conj(Ghat)
//                (cosine transform of the quadrant rows), summed over the
//                chunk's planes (the waves of a workgroup take the planes in
//                turn, their sums added in LDS in wave order), added to St_b.
//   k_adj_t2_cols / k_adj_t2_rows: three type-2 fine grids per frequency
//                (plain, kx- and ky-weighted spectra), deconvolved and
//                zero-padded, inverse FFT along y then x.
//   k_adj_interp: per relay sample, w x w gather from the three grids of
//                every frequency of the chunk (the waves of a workgroup take
//                the frequencies in turn); grad_P written, grad_xy summed over
//                frequencies in a fixed order.
#include "kernels.hpp"
#include "wavefft.hpp"

namespace nursd {

__device__ __forceinline__ double adj_dist(double x, double y, double z) {
    const double d2 = x * x + y * y + z * z;
    float inv;
    return sqrt_f64(d2, &inv);
}

__device__ __forceinline__ float2 adj_phase(double d, double foc) {
    const double cyc = d * foc;
    const float fr = (float)(cyc - rint(cyc));
    float s, c;
    sincos_cycles(fr, &s, &c);
    return make_float2(c, s);
}

template <int M>
constexpr int adj_row_waves() { return M >= 1024 ? 8 : 16; }

template <int M>
__global__ __launch_bounds__(adj_row_waves<M>() * 64) void k_adj_rows(AdjArgs a) {
    using F = WaveFFT<M>;
    constexpr int H = M / 2, E = F::E, LPW = F::LPW, NW = adj_row_waves<M>();
    constexpr int SCRP = (F::SCR > LPW * M ? F::SCR : LPW * M) + 1;
    constexpr int RB = NW * LPW;
    extern __shared__ float2 sm[];          // [NW][SCRP], twiddles M
    float2* tws = sm + NW * SCRP;
    for (int i = threadIdx.x; i < M; i += NW * 64) tws[i] = a.tw_m[i];
    const int zl = blockIdx.y;
    const int iz = a.g.z0 + zl;
    const int iy0 = blockIdx.x * RB;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nx = a.nx, ny = a.ny;
    const double z = a.g.z[iz];
    float2 gv[F::NV];
    double dist[F::NV];
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
        const int iy = iy0 + wave * LPW + q;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int n = lane + 64 * e;
            // grid column m is window column (m + (nx q)/2) / q when that divides
            const int m = n < H ? n : n - M;
            const int t = m + (nx * a.q) / 2;
            const int ix = (t >= 0 && t % a.q == 0) ? t / a.q : -1;
            const int sl = q * E + e;
            gv[sl] = make_float2(0.f, 0.f);
            dist[sl] = 0.0;
            if (iy < ny && ix >= 0 && ix < nx) {
                gv[sl] = a.gV[((size_t)iz * ny + iy) * nx + ix];
                const double x = a.xc + m * a.g.dx;
                const double y = a.yc + (iy * a.q - (ny * a.q) / 2) * a.g.dy;
                dist[sl] = adj_dist(x - a.xp0, y - a.xp1, z - a.xp2);
            }
        }
    }
    float2* scr = sm + wave * SCRP;
    for (int b = a.g.b0; b < a.g.b0 + a.g.nb; ++b) {
        const int p = (b - a.g.b0) * a.g.nzc + zl;
        const double foc = a.g.f[b] / kC;
        float2 v[F::NV];
#pragma unroll
        for (int sl = 0; sl < F::NV; ++sl) v[sl] = cmulc(gv[sl], adj_phase(dist[sl], foc));
        __syncthreads();                     // previous frequency's staging has been stored
        F::template nat_to_perm<false>(v, scr, tws, lane);
#pragma unroll
        for (int h = 0; h < F::GPL; ++h)
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                int q;
                const int k = F::perm_k(lane, h, d, q);
                scr[q * M + k] = v[h * 8 + d];
            }
        __syncthreads();
        float2* Rt = a.Rt + (size_t)p * M * ny;
        for (int i = threadIdx.x; i < M * RB; i += NW * 64) {
            const int kx = i / RB, j = i % RB;
            if (iy0 + j < ny) Rt[(size_t)kx * ny + iy0 + j] = sm[(j / LPW) * SCRP + (j % LPW) * M + kx];
        }
    }
}

constexpr int kAdjColWaves = 8;

template <int M>
__global__ __launch_bounds__(kAdjColWaves * 64) void k_adj_cols(AdjArgs a) {
    using F = WaveFFT<M>;
    constexpr int H = M / 2, E = F::E, LPW = F::LPW;
    static_assert(kAdjColWaves * F::NV * 64 <= kAdjColWaves * F::SCR, "reduction must fit the scratch");
    extern __shared__ float2 sm[];          // [waves][SCR] (then the partial sums), twiddles M
    float2* tws = sm + kAdjColWaves * F::SCR;
    for (int i = threadIdx.x; i < M; i += kAdjColWaves * 64) tws[i] = a.tw_m[i];
    __syncthreads();
    const int fb = blockIdx.y;
    const int b = a.g.b0 + fb;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // one group of LPW kx lines per workgroup (kx0 <= H by the grid); its
    // waves take the chunk's planes in turn and their sums meet in LDS
    const int kx0 = blockIdx.x * LPW;
    float2* scr = sm + wave * F::SCR;
    const int ny = a.ny, hq = (ny * a.q) / 2;
    float2 acc[2][F::NV];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int i = 0; i < F::NV; ++i) acc[sd][i] = make_float2(0.f, 0.f);
    for (int zl = wave; zl < a.g.nzc; zl += kAdjColWaves) {
        const int p = fb * a.g.nzc + zl;
        const float2* Bt = a.Bt + (size_t)p * (H + 1) * a.BS;
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
        const float2* Rt = a.Rt + (size_t)p * M * ny;
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            float2 v[F::NV];
#pragma unroll
            for (int q = 0; q < LPW; ++q) {
                const int kx = kx0 + q;
                const int s = sd ? ((M - kx) & (M - 1)) : kx;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int n = lane + 64 * e;
                    // grid row m is window row (m + (ny q)/2) / q when that divides
                    const int t = (n < H ? n : n - M) + hq;
                    const int iy = (t >= 0 && t % a.q == 0) ? t / a.q : -1;
                    v[q * E + e] = (kx <= H && iy >= 0 && iy < ny) ? Rt[(size_t)s * ny + iy] : make_float2(0.f, 0.f);
                }
            }
            F::template nat_to_perm<false>(v, scr, tws, lane);
#pragma unroll
            for (int i = 0; i < F::NV; ++i) acc[sd][i] = cadd(acc[sd][i], cmulc(v[i], g[i]));
        }
    }
    float2* St = a.St + (size_t)b * M * M;
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
        __syncthreads();                    // scratch free (FFTs or the previous side done)
#pragma unroll
        for (int i = 0; i < F::NV; ++i) sm[(wave * F::NV + i) * 64 + lane] = acc[sd][i];
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int h = 0; h < F::GPL; ++h)
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    const int i = h * 8 + d;
                    float2 t = sm[i * 64 + lane];
                    for (int w = 1; w < kAdjColWaves; ++w) t = cadd(t, sm[(w * F::NV + i) * 64 + lane]);
                    int q;
                    const int k = F::perm_k(lane, h, d, q);
                    const int kx = kx0 + q;
                    const int s = sd ? ((M - kx) & (M - 1)) : kx;
                    if (kx > H || (sd && s == kx)) continue;
                    float2* o = St + (size_t)s * M + k;
                    *o = a.first ? t : cadd(*o, t);
                }
        }
    }
}

// Three type-2 spectra per frequency: q = 0 plain, 1 times j 2 pi kx / Lx,
// 2 times j 2 pi ky / Ly; deconvolved ((-1)^k / phihat(k) per axis), scaled
// by M^-2, zero-padded to MF and inverse-transformed along y.
template <int MF>
__global__ __launch_bounds__(8 * 64) void k_adj_t2_cols(AdjArgs a) {
    using G = WaveFFT<MF>;
    constexpr int EG = G::E, LPW = G::LPW;
    extern __shared__ float2 sm[];          // [8][SCR], twiddles MF
    float2* tws = sm + 8 * G::SCR;
    for (int i = threadIdx.x; i < MF; i += 8 * 64) tws[i] = a.tw_f[i];
    __syncthreads();
    const int M = MF / 2, H = M / 2;
    const int fb = blockIdx.y, qk = blockIdx.z;
    const int b = a.g.b0 + fb;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int s0 = (blockIdx.x * 8 + wave) * LPW;
    if (s0 >= M) return;
    const float2* St = a.St + (size_t)b * M * M;
    const float inv_m2 = 1.0f / ((float)M * (float)M);
    float2 v[G::NV];
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
        const int s = s0 + q;
        const int kxs = s < H ? s : s - M;
        const float fx = a.dec[s] * inv_m2;
#pragma unroll
        for (int e = 0; e < EG; ++e) {
            const int n = lane + 64 * e;
            const int ky = n < H ? n : (n >= MF - H ? n - MF : 1 << 20);
            float2 val = make_float2(0.f, 0.f);
            if (ky != (1 << 20)) {
                const int km = ky & (M - 1);
                val = cscale(St[(size_t)s * M + km], fx * a.dec[km]);
                if (qk == 1) val = cscale(make_float2(-val.y, val.x), a.kscale_x * (float)kxs);
                if (qk == 2) val = cscale(make_float2(-val.y, val.x), a.kscale_y * (float)ky);
            }
            v[q * EG + e] = val;
        }
    }
    G::template nat_to_perm<true>(v, sm + wave * G::SCR, tws, lane);
    float2* T3 = a.T3 + ((size_t)fb * 3 + qk) * M * MF;
#pragma unroll
    for (int h = 0; h < G::GPL; ++h)
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            int q;
            const int jy = G::perm_k(lane, h, d, q);
            T3[(size_t)(s0 + q) * MF + jy] = v[h * 8 + d];
        }
}

template <int MF>
__global__ __launch_bounds__(8 * 64) void k_adj_t2_rows(AdjArgs a) {
    using G = WaveFFT<MF>;
    constexpr int EG = G::E, LPW = G::LPW;
    constexpr int SCRP = (G::SCR > LPW * MF ? G::SCR : LPW * MF) + 1;
    constexpr int RB = 8 * LPW;
    extern __shared__ float2 sm[];          // [8][SCRP], twiddles MF
    float2* tws = sm + 8 * SCRP;
    for (int i = threadIdx.x; i < MF; i += 8 * 64) tws[i] = a.tw_f[i];
    const int M = MF / 2, H = M / 2;
    const int fb = blockIdx.y, qk = blockIdx.z;
    const int jy0 = a.relay_row_lo + blockIdx.x * RB;
    if (jy0 > a.relay_row_hi) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const float2* T3 = a.T3 + ((size_t)fb * 3 + qk) * M * MF;
    for (int i = threadIdx.x; i < MF * RB; i += 8 * 64) {
        const int n = i / RB, j = i % RB;
        const int jy = (jy0 + j) & (MF - 1);
        float2 val = make_float2(0.f, 0.f);
        if (n < H) val = T3[(size_t)n * MF + jy];
        else if (n >= MF - H) val = T3[(size_t)(n - MF + M) * MF + jy];
        sm[(j / LPW) * SCRP + (j % LPW) * MF + n] = val;
    }
    __syncthreads();
    float2* rows = sm + wave * SCRP;
    float2 v[G::NV];
#pragma unroll
    for (int q = 0; q < LPW; ++q)
#pragma unroll
        for (int e = 0; e < EG; ++e) v[q * EG + e] = rows[q * MF + lane + 64 * e];
    G::template nat_to_perm<true>(v, rows, tws, lane);
    float2* G3 = a.G3 + ((size_t)fb * 3 + qk) * MF * MF;
#pragma unroll
    for (int h = 0; h < G::GPL; ++h)
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            int q;
            const int jx = G::perm_k(lane, h, d, q);
            const int jy = (jy0 + wave * LPW + q) & (MF - 1);
            G3[(size_t)jy * MF + jx] = v[h * 8 + d];
        }
}

__device__ __forceinline__ float es_a(float z, float beta) {
    const float t = fmaxf(1.0f - z * z, 0.0f);
    return __expf(beta * (sqrtf(t) - 1.0f));
}

constexpr int kAdjInterpWaves = 8;

// One workgroup per 64 relay samples; its waves take the chunk's frequencies
// in turn (grad_P per frequency), and the position gradients of the waves are
// added in LDS in wave order.
__global__ __launch_bounds__(kAdjInterpWaves * 64) void k_adj_interp(AdjArgs a) {
    __shared__ float2 gpart[kAdjInterpWaves][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int l = blockIdx.x * 64 + lane;
    const bool live = l < a.L;
    float gx = 0.f, gy = 0.f;
    if (live) {
        const int MF = a.Mf;
        const double hw = 0.5 * a.w;
        const double tx = ((double)a.relay[2 * l] - a.cx) / a.g.dx * 2.0 + MF / 2;
        const double ty = ((double)a.relay[2 * l + 1] - a.cy) / a.g.dy * 2.0 + MF / 2;
        const int ix0 = (int)ceil(tx - hw), iy0 = (int)ceil(ty - hw);
        const float fx = (float)(tx - ix0), fy = (float)(ty - iy0);
        const float ihw = (float)(1.0 / hw);
        float wx[8], wy[8];
        int col[8], rowoff[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            wx[i] = i < a.w ? es_a(((float)i - fx) * ihw, a.beta) : 0.f;
            wy[i] = i < a.w ? es_a(((float)i - fy) * ihw, a.beta) : 0.f;
            col[i] = (ix0 + i) & (MF - 1);
            rowoff[i] = ((iy0 + i) & (MF - 1)) * MF;
        }
        const int nq = a.grad_xy ? 3 : 1;
        const float wl = a.wts ? a.wts[l] : 1.0f;
        for (int fb = wave; fb < a.g.nb; fb += kAdjInterpWaves) {
            const int b = a.g.b0 + fb;
            float2 val[3];
            for (int qk = 0; qk < nq; ++qk) {
                const float2* G3 = a.G3 + ((size_t)fb * 3 + qk) * MF * MF;
                float2 sum = make_float2(0.f, 0.f);
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    if (j >= a.w) break;
                    const float2* row = G3 + rowoff[j];
                    float2 r = make_float2(0.f, 0.f);
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        if (i >= a.w) break;
                        const float2 g = row[col[i]];
                        r.x = fmaf(wx[i], g.x, r.x);
                        r.y = fmaf(wx[i], g.y, r.y);
                    }
                    sum.x = fmaf(wy[j], r.x, sum.x);
                    sum.y = fmaf(wy[j], r.y, sum.y);
                }
                val[qk] = sum;
            }
            // the forward used w_l P_l: both gradients carry the weight
            a.grad_P[(size_t)b * a.L + l] = cscale(val[0], wl);
            if (a.grad_xy) {
                const float2 pv = a.P[(size_t)b * a.L + l];
                gx += wl * (pv.x * val[1].x + pv.y * val[1].y);     // Re(conj(w P) D)
                gy += wl * (pv.x * val[2].x + pv.y * val[2].y);
            }
        }
    }
    if (!a.grad_xy) return;                 // uniform: no barrier below is skipped by part of the block
    gpart[wave][lane] = make_float2(gx, gy);
    __syncthreads();
    if (wave != 0 || !live) return;
    float2 t = a.first_b ? make_float2(0.f, 0.f) : make_float2(a.grad_xy[2 * l], a.grad_xy[2 * l + 1]);
#pragma unroll
    for (int w = 0; w < kAdjInterpWaves; ++w) t = cadd(t, gpart[w][lane]);
    a.grad_xy[2 * l] = t.x;
    a.grad_xy[2 * l + 1] = t.y;
}

template <typename Args>
static hipError_t launch_a(void (*k)(Args), dim3 grid, int threads, size_t sh, hipStream_t s, const Args& a) {
    if (sh > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, grid, dim3(threads), sh, s, a);
    return hipGetLastError();
}

template <int M>
static hipError_t adj_planes_impl(const AdjArgs& a, hipStream_t s) {
    using F = WaveFFT<M>;
    constexpr int NW = adj_row_waves<M>();
    constexpr int SCRP = (F::SCR > F::LPW * M ? F::SCR : F::LPW * M) + 1;
    constexpr int RB = NW * F::LPW;
    hipError_t e = launch_a(k_adj_rows<M>, dim3((a.ny + RB - 1) / RB, a.g.nzc), NW * 64,
                            (size_t)(NW * SCRP + M) * sizeof(float2), s, a);
    if (e != hipSuccess) return e;
    return launch_a(k_adj_cols<M>, dim3((M / 2 + 1 + F::LPW - 1) / F::LPW, a.g.nb), kAdjColWaves * 64,
                    (size_t)(kAdjColWaves * F::SCR + M) * sizeof(float2), s, a);
}

hipError_t launch_adjoint_planes(const AdjArgs& a, hipStream_t s) {
    switch (a.M) {
        case 64: return adj_planes_impl<64>(a, s);
        case 128: return adj_planes_impl<128>(a, s);
        case 256: return adj_planes_impl<256>(a, s);
        case 512: return adj_planes_impl<512>(a, s);
        case 1024: return adj_planes_impl<1024>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int MF>
static hipError_t adj_t2_impl(const AdjArgs& a, hipStream_t s) {
    using G = WaveFFT<MF>;
    const int M = MF / 2;
    const int nq = a.grad_xy ? 3 : 1;
    hipError_t e = launch_a(k_adj_t2_cols<MF>, dim3((M + 8 * G::LPW - 1) / (8 * G::LPW), a.g.nb, nq), 8 * 64,
                            (size_t)(8 * G::SCR + MF) * sizeof(float2), s, a);
    if (e != hipSuccess) return e;
    constexpr int SCRP = (G::SCR > G::LPW * MF ? G::SCR : G::LPW * MF) + 1;
    constexpr int RB = 8 * G::LPW;
    e = launch_a(k_adj_t2_rows<MF>, dim3((MF + RB - 1) / RB, a.g.nb, nq), 8 * 64,
                 (size_t)(8 * SCRP + MF) * sizeof(float2), s, a);
    if (e != hipSuccess) return e;
    return launch_a(k_adj_interp, dim3((a.L + 63) / 64), kAdjInterpWaves * 64, 0, s, a);
}

hipError_t launch_adjoint_type2(const AdjArgs& a, hipStream_t s) {
    switch (a.Mf) {
        case 128: return adj_t2_impl<128>(a, s);
        case 256: return adj_t2_impl<256>(a, s);
        case 512: return adj_t2_impl<512>(a, s);
        case 1024: return adj_t2_impl<1024>(a, s);
        case 2048: return adj_t2_impl<2048>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace nursd
