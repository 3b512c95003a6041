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
#include "fft.hpp"
#include "kernels.hpp"

namespace nursd {

constexpr int kRsdThreads = 512;
constexpr int kRsdLines = 8;

// e^{+j 2 pi (r f / c)} / r for r = sqrt(r2); the cycle count r f / c is
// formed in FP64 and reduced to [-1/2, 1/2] before the FP32 sin/cos.
__device__ __forceinline__ float2 rsd_kernel(double r2, double f_over_c) {
    const float r0 = sqrtf((float)r2);
    const double r = (double)r0 + (r2 - (double)r0 * (double)r0) * (double)(0.5f / r0);
    const double cyc = r * f_over_c;
    const float fr = (float)(cyc - rint(cyc));
    float s, c;
    sincospif(2.0f * fr, &s, &c);
    const float ir = 1.0f / (float)r;
    return make_float2(c * ir, s * ir);
}

// e^{+j 2 pi d f / c} for a precomputed distance d.
__device__ __forceinline__ float2 phase_of(double d, double f_over_c) {
    const double cyc = d * f_over_c;
    const float fr = (float)(cyc - rint(cyc));
    float s, c;
    sincospif(2.0f * fr, &s, &c);
    return make_float2(c, s);
}

__device__ __forceinline__ double dist3(double x, double y, double z) {
    const double d2 = x * x + y * y + z * z;
    const float d0 = sqrtf((float)d2);
    return (double)d0 + (d2 - (double)d0 * (double)d0) * (double)(0.5f / d0);
}

__device__ __forceinline__ void plane_of(const ChunkGeom& g, int p, int& b, int& iz) {
    b = g.b0 + p / g.nzc;
    iz = g.z0 + p % g.nzc;
}

template <int M>
__global__ __launch_bounds__(kRsdThreads) void k_kernel_rows(P1Args a) {
    extern __shared__ float2 sm[];      // [kRsdLines][M]
    constexpr int H = M / 2;
    const int p = blockIdx.y;
    int b, iz;
    plane_of(a.g, p, b, iz);
    const double foc = a.g.f[b] / kC;
    const double z = a.g.z[iz];
    const double px = a.g.pitch_x ? a.g.pitch_x[iz] : a.g.dx;
    const double py = a.g.pitch_y ? a.g.pitch_y[iz] : a.g.dy;
    const int my0 = blockIdx.x * kRsdLines;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int my = my0 + wave;
    float2* line = sm + wave * M;
    if (my <= H) {
        const double ry = my * py;
        const double ryz = fma(ry, ry, z * z);
        for (int n = lane; n <= H; n += 64) {
            const double rx = n * px;
            const float2 g = rsd_kernel(fma(rx, rx, ryz), foc);
            line[n] = g;
            if (n > 0 && n < H) line[M - n] = g;
        }
    } else {
        for (int n = lane; n < M; n += 64) line[n] = make_float2(0.f, 0.f);
    }
    __syncthreads();
    fft_lines<M, 64, false>(sm, M, kRsdLines, a.tw);
    float2* Bt = a.Bt + (size_t)p * (H + 1) * a.BS;
    for (int i = tid; i < (H + 1) * kRsdLines; i += kRsdThreads) {
        const int kx = i / kRsdLines, l = i % kRsdLines;
        if (my0 + l <= H) Bt[(size_t)kx * a.BS + my0 + l] = sm[l * M + kx];
    }
}

template <int M>
__global__ __launch_bounds__(kRsdThreads) void k_propagate_cols(P2Args a) {
    extern __shared__ float2 sm[];      // [2 * kRsdLines][M]: +kx lines, then -kx lines
    constexpr int H = M / 2;
    const int p = blockIdx.y;
    int b, iz;
    plane_of(a.g, p, b, iz);
    const int kx0 = blockIdx.x * kRsdLines;
    const int tid = threadIdx.x;
    const float2* Bt = a.Bt + (size_t)p * (H + 1) * a.BS;
    for (int i = tid; i < kRsdLines * M; i += kRsdThreads) {
        const int l = i / M, n = i % M;
        const int kx = kx0 + l;
        const int d = n <= H ? n : M - n;
        sm[i] = kx <= H ? Bt[(size_t)kx * a.BS + d] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    fft_lines<M, 64, false>(sm, M, kRsdLines, a.tw);          // Ghat[kx][ky]
    const float2* Ub = a.U + (size_t)b * M * M;
    for (int i = tid; i < kRsdLines * M; i += kRsdThreads) {
        const int l = i / M, ky = i % M;
        const int kx = kx0 + l;
        if (kx <= H) {
            const float2 g = sm[i];
            const int s2 = (M - kx) & (M - 1);
            sm[(kRsdLines + l) * M + ky] = s2 != kx ? cmul(Ub[(size_t)s2 * M + ky], g) : make_float2(0.f, 0.f);
            sm[i] = cmul(Ub[(size_t)kx * M + ky], g);
        }
    }
    __syncthreads();
    fft_lines<M, kRsdThreads / (2 * kRsdLines), true>(sm, M, 2 * kRsdLines, a.tw);
    float2* Yt = a.Yt + (size_t)p * a.ny * M;
    const int half = a.ny / 2;
    for (int i = tid; i < a.ny * 2 * kRsdLines; i += kRsdThreads) {
        const int iy = i / (2 * kRsdLines), q = i % (2 * kRsdLines);
        const int l = q % kRsdLines;
        const int kx = kx0 + l;
        if (kx > H) continue;
        const int s = q < kRsdLines ? kx : ((M - kx) & (M - 1));
        if (q >= kRsdLines && s == kx) continue;
        const int my = (iy - half) & (M - 1);
        Yt[(size_t)iy * M + s] = sm[q * M + my];
    }
}

constexpr int kP3MaxVox = 8;   // voxels per thread: kRsdLines * nx / kRsdThreads <= 8 (nx <= 512)

template <int M>
__global__ __launch_bounds__(kRsdThreads) void k_propagate_rows(P3Args a) {
    extern __shared__ float2 sm[];      // [kRsdLines][M]
    const int zl = blockIdx.y;
    const int iz = a.g.z0 + zl;
    const int iy0 = blockIdx.x * kRsdLines;
    const int tid = threadIdx.x;
    const int nx = a.nx;
    const int nvox = kRsdLines * nx;
    const double z = a.g.z[iz];
    const double px = a.g.pitch_x ? a.g.pitch_x[iz] : a.g.dx;
    const double py = a.g.pitch_y ? a.g.pitch_y[iz] : a.g.dy;
    double d[kP3MaxVox];
    float2 acc[kP3MaxVox];
    const size_t plane_off = (size_t)iz * a.ny * nx;
#pragma unroll
    for (int k = 0; k < kP3MaxVox; ++k) {
        const int v = tid + k * kRsdThreads;
        const int l = v / nx, ix = v % nx;
        const int iy = iy0 + l;
        acc[k] = make_float2(0.f, 0.f);
        d[k] = 0.0;
        if (v < nvox && iy < a.ny) {
            const double x = a.xc + (ix - nx / 2) * px;
            const double y = a.yc + (iy - a.ny / 2) * py;
            d[k] = dist3(x - a.xp0, y - a.xp1, z - a.xp2);
            if (!a.first) {
                const size_t o = plane_off + (size_t)iy * nx + ix;
                if (a.coherent) acc[k] = a.V[o];
                else acc[k].x = a.I[o];
            }
        }
    }
    for (int b = a.g.b0; b < a.g.b0 + a.g.nb; ++b) {
        const int p = (b - a.g.b0) * a.g.nzc + zl;
        const float2* Yt = a.Yt + (size_t)p * a.ny * M;
        for (int i = tid; i < kRsdLines * M; i += kRsdThreads) {
            const int l = i / M, c = i % M;
            sm[i] = (iy0 + l < a.ny) ? Yt[(size_t)(iy0 + l) * M + c] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        fft_lines<M, 64, true>(sm, M, kRsdLines, a.tw);
        const double foc = a.g.f[b] / kC;
#pragma unroll
        for (int k = 0; k < kP3MaxVox; ++k) {
            const int v = tid + k * kRsdThreads;
            if (v < nvox) {
                const int l = v / nx, ix = v % nx;
                const float2 val = sm[l * M + ((ix - nx / 2) & (M - 1))];
                if (a.coherent) {
                    const float2 ph = phase_of(d[k], foc);
                    acc[k] = cadd(acc[k], cmul(ph, val));
                } else {
                    acc[k].x += sqrtf(val.x * val.x + val.y * val.y);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kP3MaxVox; ++k) {
        const int v = tid + k * kRsdThreads;
        const int l = v / nx, ix = v % nx;
        const int iy = iy0 + l;
        if (v < nvox && iy < a.ny) {
            const size_t o = plane_off + (size_t)iy * nx + ix;
            if (a.coherent) {
                if (a.V) a.V[o] = acc[k];
                if (a.last && a.I) a.I[o] = sqrtf(acc[k].x * acc[k].x + acc[k].y * acc[k].y);
            } else {
                a.I[o] = acc[k].x;
            }
        }
    }
}

template <int M, typename Args>
static hipError_t launch_rsd(void (*k)(Args), dim3 grid, size_t sh, hipStream_t s, const Args& a) {
    if (sh > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, grid, dim3(kRsdThreads), sh, s, a);
    return hipGetLastError();
}

#define NURSD_SWITCH_M(M_, CALL)                           \
    switch (M_) {                                          \
        case 16: { constexpr int MM = 16; CALL; }          \
        case 32: { constexpr int MM = 32; CALL; }          \
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
        dim3 grid((MM / 2 + 1 + kRsdLines - 1) / kRsdLines, planes);
        return launch_rsd<MM>(k_kernel_rows<MM>, grid, (size_t)kRsdLines * MM * sizeof(float2), s, a);
    })
}

hipError_t launch_propagate_cols(const P2Args& a, hipStream_t s) {
    const int planes = a.g.nb * a.g.nzc;
    NURSD_SWITCH_M(a.M, {
        dim3 grid((MM / 2 + 1 + kRsdLines - 1) / kRsdLines, planes);
        return launch_rsd<MM>(k_propagate_cols<MM>, grid, (size_t)2 * kRsdLines * MM * sizeof(float2), s, a);
    })
}

hipError_t launch_propagate_rows(const P3Args& a, hipStream_t s) {
    if (a.nx * kRsdLines > kP3MaxVox * kRsdThreads) return hipErrorInvalidValue;
    NURSD_SWITCH_M(a.M, {
        dim3 grid((a.ny + kRsdLines - 1) / kRsdLines, a.g.nzc);
        return launch_rsd<MM>(k_propagate_rows<MM>, grid, (size_t)kRsdLines * MM * sizeof(float2), s, a);
    })
}

}  // namespace nursd
