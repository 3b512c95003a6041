// Register-resident FFT of one 64-lane wavefront (CDNA4), N = E * 64 points.
//
// Layouts (lane = threadIdx.x & 63):
//   natural:  v[q*E + e] = x_q[lane + 64 e]   (q < LPW lines per wave)
//   permuted: v[h*8 + d] = X_q[k1 + E c + 8 E d], where the group index
//             gi = lane + 64 h decodes as q = gi / (8E), k1 = (gi % 8E) / 8,
//             c = gi % 8.
// The transform is N = E x 64 with the 64-point part split 8 x 8:
//   E-point DFT in registers, twiddle W_N^{lane k1}, transpose through LDS,
//   8-point DFT, twiddle W_64^{a c}, transpose, 8-point DFT.
// nat_to_perm runs these steps; perm_to_nat runs the adjoint steps in reverse
// order, so a forward nat_to_perm followed by an inverse perm_to_nat never
// needs the permutation undone (pointwise products work in either order).
// The two LDS transposes use a padded [8][9] tile per (line, k1) so lane
// strides are not multiples of the bank width.  All exchange traffic stays
// inside one wavefront: LDS operations of a wave execute in order, so only
// a compiler-level wave fence separates the write and read phases.
#pragma once
#include "fft.hpp"

#ifndef NURSD_WFFT_RP
#define NURSD_WFFT_RP 9
#endif

namespace nursd {

#define NURSD_WAVE_SYNC()                                   \
    do {                                                    \
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); \
        __builtin_amdgcn_wave_barrier();                    \
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront"); \
    } while (0)

// cos/sin(2 pi k / 16), k = 0..7 and cos/sin(2 pi k / 32), k = 0..15
__device__ constexpr float kC16[8] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                                      0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f};
__device__ constexpr float kS16[8] = {0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
                                      1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f};
__device__ constexpr float kC32[16] = {1.0f, 0.98078528040323043f, 0.92387953251128674f, 0.83146961230254524f,
                                       0.70710678118654752f, 0.55557023301960218f, 0.38268343236508977f,
                                       0.19509032201612827f, 0.0f, -0.19509032201612827f, -0.38268343236508977f,
                                       -0.55557023301960218f, -0.70710678118654752f, -0.83146961230254524f,
                                       -0.92387953251128674f, -0.98078528040323043f};
__device__ constexpr float kS32[16] = {0.0f, 0.19509032201612827f, 0.38268343236508977f, 0.55557023301960218f,
                                       0.70710678118654752f, 0.83146961230254524f, 0.92387953251128674f,
                                       0.98078528040323043f, 1.0f, 0.98078528040323043f, 0.92387953251128674f,
                                       0.83146961230254524f, 0.70710678118654752f, 0.55557023301960218f,
                                       0.38268343236508977f, 0.19509032201612827f};

// In-register DFT of R = 1..32 points (forward e^{-}, inverse e^{+}).
// LO: the inputs v[R/2..R-1] are zero (R >= 4) and are not read.
template <int R, bool INV, bool LO = false>
__device__ __forceinline__ void dft_reg(float2* v) {
    static_assert(!LO || R >= 4, "zero upper half needs at least 4 points");
    if constexpr (R == 1) {
        return;
    } else if constexpr (LO && R == 4) {
        dft4_lo<INV>(v);
    } else if constexpr (LO && R == 8) {
        dft8_lo<INV>(v);
    } else if constexpr (R <= 8) {
        dftR<R, INV>(v);
    } else {
        float2 ev[R / 2], od[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            ev[i] = LO && 2 * i >= R / 2 ? make_float2(0.f, 0.f) : v[2 * i];
            od[i] = LO && 2 * i + 1 >= R / 2 ? make_float2(0.f, 0.f) : v[2 * i + 1];
        }
        dft_reg<R / 2, INV, LO>(ev);
        dft_reg<R / 2, INV, LO>(od);
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            const float c = R == 16 ? kC16[k] : kC32[k];
            const float s = R == 16 ? kS16[k] : kS32[k];
            const float2 w = make_float2(c, INV ? s : -s);
            const float2 t = cmul(od[k], w);
            v[k] = cadd(ev[k], t);
            v[k + R / 2] = csub(ev[k], t);
        }
    }
}

template <bool INV>
__device__ __forceinline__ float2 twiddle(float2 v, float2 w) {
    return INV ? cmulc(v, w) : cmul(v, w);
}

template <int N>
struct WaveFFT {
    static_assert(N >= 64 && N <= 2048 && (N & (N - 1)) == 0, "wave FFT size");
    static constexpr int E = N / 64;
    static constexpr int LPW = N >= 512 ? 1 : 512 / N;   // lines per wave
    static constexpr int GPL = E >= 8 ? E / 8 : 1;       // 8-point groups per lane
    static constexpr int NV = E * LPW;                   // values per lane (== 8 * GPL)
    // Exchange tile of one (line, k1): 8 rows of RP float2 (RP > 8 keeps the
    // lane strides off multiples of the bank count); BP per tile.
    static constexpr int RP = NURSD_WFFT_RP, BP = 8 * RP;
    static constexpr int SCR = LPW * E * BP;             // LDS scratch per wave (float2)
    // Twiddle entries the transforms read: tw[lane k1] (lane < 64, k1 < E)
    // and tw[E a c] (a, c < 8), neither of which wraps; a kernel that stages
    // the table in LDS needs only these.
    static constexpr int TWN = (63 * (E - 1) > 49 * E ? 63 * (E - 1) : 49 * E) + 1;
    static_assert(NV == 8 * GPL, "layout");

    __device__ static __forceinline__ void decode(int gi, int& q, int& k1, int& x) {
        q = gi / (8 * E);
        const int r = gi % (8 * E);
        k1 = r >> 3;
        x = r & 7;
    }
    // natural index (and line) of permuted slot (h, d) of this lane
    __device__ static __forceinline__ int perm_k(int lane, int h, int d, int& q) {
        int k1, c;
        decode(lane + 64 * h, q, k1, c);
        return k1 + E * c + 8 * E * d;
    }

    // LO (one line per wave, E >= 4): the inputs n >= N/2 (slots e >= E/2)
    // are zero and are not read.
    template <bool INV, bool LO = false>
    __device__ static __forceinline__ void nat_to_perm(float2* v, float2* scr, const float2* __restrict__ tw,
                                                       int lane) {
        static_assert(!LO || (LPW == 1 && E >= 4), "zero upper half needs one line of at least 256 points");
        const int a = lane & 7, b = lane >> 3;
#pragma unroll
        for (int q = 0; q < LPW; ++q) {
            float2* y = v + q * E;
            dft_reg<E, INV, LO>(y);
#pragma unroll
            for (int k1 = 1; k1 < E; ++k1) y[k1] = twiddle<INV>(y[k1], tw[(lane * k1) & (N - 1)]);
        }
        NURSD_WAVE_SYNC();
#pragma unroll
        for (int q = 0; q < LPW; ++q)
#pragma unroll
            for (int k1 = 0; k1 < E; ++k1) scr[(q * E + k1) * BP + a * RP + b] = v[q * E + k1];
        NURSD_WAVE_SYNC();
#pragma unroll
        for (int h = 0; h < GPL; ++h) {
            int q, k1, aa;
            decode(lane + 64 * h, q, k1, aa);
            const int base = (q * E + k1) * BP + aa * RP;
            float2* t = v + h * 8;
#pragma unroll
            for (int bb = 0; bb < 8; ++bb) t[bb] = scr[base + bb];
            dft_reg<8, INV>(t);
#pragma unroll
            for (int c = 1; c < 8; ++c) t[c] = twiddle<INV>(t[c], tw[(E * aa * c) & (N - 1)]);
        }
        NURSD_WAVE_SYNC();
#pragma unroll
        for (int h = 0; h < GPL; ++h) {
            int q, k1, aa;
            decode(lane + 64 * h, q, k1, aa);
            const int base = (q * E + k1) * BP + aa;
#pragma unroll
            for (int c = 0; c < 8; ++c) scr[base + c * RP] = v[h * 8 + c];
        }
        NURSD_WAVE_SYNC();
#pragma unroll
        for (int h = 0; h < GPL; ++h) {
            int q, k1, c;
            decode(lane + 64 * h, q, k1, c);
            const int base = (q * E + k1) * BP + c * RP;
            float2* w = v + h * 8;
#pragma unroll
            for (int aa = 0; aa < 8; ++aa) w[aa] = scr[base + aa];
            dft_reg<8, INV>(w);
        }
        NURSD_WAVE_SYNC();
    }

    template <bool INV>
    __device__ static __forceinline__ void perm_to_nat(float2* v, float2* scr, const float2* __restrict__ tw,
                                                       int lane) {
#pragma unroll
        for (int h = 0; h < GPL; ++h) dft_reg<8, INV>(v + h * 8);
        NURSD_WAVE_SYNC();
#pragma unroll
        for (int h = 0; h < GPL; ++h) {
            int q, k1, c;
            decode(lane + 64 * h, q, k1, c);
            const int base = (q * E + k1) * BP + c * RP;
#pragma unroll
            for (int aa = 0; aa < 8; ++aa) scr[base + aa] = v[h * 8 + aa];
        }
        NURSD_WAVE_SYNC();
#pragma unroll
        for (int h = 0; h < GPL; ++h) {
            int q, k1, aa;
            decode(lane + 64 * h, q, k1, aa);
            const int base = (q * E + k1) * BP + aa;
            float2* u = v + h * 8;
#pragma unroll
            for (int c = 0; c < 8; ++c) u[c] = scr[base + c * RP];
#pragma unroll
            for (int c = 1; c < 8; ++c) u[c] = twiddle<INV>(u[c], tw[(E * aa * c) & (N - 1)]);
            dft_reg<8, INV>(u);
        }
        NURSD_WAVE_SYNC();
#pragma unroll
        for (int h = 0; h < GPL; ++h) {
            int q, k1, aa;
            decode(lane + 64 * h, q, k1, aa);
            const int base = (q * E + k1) * BP + aa * RP;
#pragma unroll
            for (int bb = 0; bb < 8; ++bb) scr[base + bb] = v[h * 8 + bb];
        }
        NURSD_WAVE_SYNC();
        const int a = lane & 7, b = lane >> 3;
#pragma unroll
        for (int q = 0; q < LPW; ++q) {
            float2* y = v + q * E;
#pragma unroll
            for (int k1 = 0; k1 < E; ++k1) y[k1] = scr[(q * E + k1) * BP + a * RP + b];
#pragma unroll
            for (int k1 = 1; k1 < E; ++k1) y[k1] = twiddle<INV>(y[k1], tw[(lane * k1) & (N - 1)]);
            dft_reg<E, INV>(y);
        }
        NURSD_WAVE_SYNC();
    }
};

}  // namespace nursd
