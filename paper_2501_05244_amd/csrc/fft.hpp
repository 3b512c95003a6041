// Complex helpers and an in-LDS Stockham FFT for CDNA4 (gfx950).
//
// Lines of N = 2^n complex64 samples live in LDS; a group of TPL threads
// (one or more 64-lane wavefronts) transforms each line.  Every radix pass
// reads R samples per butterfly into registers, applies the twiddles, does
// the radix-R DFT and writes the autosorted result back in place after a
// workgroup barrier, so no second buffer is needed.  Twiddles come from a
// per-size table tw[m] = e^{-2 pi j m / N} built in float64 on the host and
// rounded once to float32.
#pragma once
#include <hip/hip_runtime.h>

namespace nursd {

struct c2 {
    float x, y;
};

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// sin and cos of 2 pi x for x in [-1/2, 1/2] (a phase already reduced to a
// fraction of a cycle in FP64) on the transcendental unit, whose argument is
// in revolutions: one instruction each, absolute error about 1.3e-7 on this
// range against float64 (a float32 library sincos is about 5e-8).
__device__ __forceinline__ void sincos_cycles(float x, float* s, float* c) {
    *s = __builtin_amdgcn_sinf(x);
    *c = __builtin_amdgcn_cosf(x);
}
// sqrt(d2) to FP64 accuracy: hardware FP32 square root and reciprocal as the
// estimate d0, then one Newton step d0 + (d2 - d0^2) / (2 d0) in FP64.  The
// reciprocal of the estimate is returned in *inv (relative error ~1e-7).
__device__ __forceinline__ double sqrt_f64(double d2, float* inv) {
    const float d0 = __builtin_amdgcn_sqrtf((float)d2);
    const float i0 = __builtin_amdgcn_rcpf(d0);
    *inv = i0;
    return (double)d0 + (d2 - (double)d0 * (double)d0) * (double)(0.5f * i0);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -j (forward) or +j (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mj(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2* v) {
    float2 a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2* v) {
    float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    float2 a2 = cadd(v[1], v[3]), a3 = mul_mj<INV>(csub(v[1], v[3]));
    v[0] = cadd(a0, a2);
    v[2] = csub(a0, a2);
    v[1] = cadd(a1, a3);
    v[3] = csub(a1, a3);
}

// dft4 of (v0, v1, 0, 0): the inputs above the first half are zero.
template <bool INV>
__device__ __forceinline__ void dft4_lo(float2* v) {
    const float2 a = v[0], b = v[1], jb = mul_mj<INV>(b);
    v[0] = cadd(a, b);
    v[1] = cadd(a, jb);
    v[2] = csub(a, b);
    v[3] = csub(a, jb);
}

// Last step of the 8-point DFT from the 4-point DFTs of the even and odd
// inputs.
template <bool INV>
__device__ __forceinline__ void dft8_join(float2* v, const float2* e, const float2* o) {
    constexpr float h = 0.70710678118654752440f;
    // w8^1 = (1 -/+ j)/sqrt2, w8^2 = -/+ j, w8^3 = (-1 -/+ j)/sqrt2
    float2 t1 = INV ? make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
                    : make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    float2 t2 = mul_mj<INV>(o[2]);
    float2 t3 = INV ? make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
                    : make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], t1);
    v[5] = csub(e[1], t1);
    v[2] = cadd(e[2], t2);
    v[6] = csub(e[2], t2);
    v[3] = cadd(e[3], t3);
    v[7] = csub(e[3], t3);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    dft4<INV>(e);
    dft4<INV>(o);
    dft8_join<INV>(v, e, o);
}

// dft8 of (v0, v1, v2, v3, 0, 0, 0, 0): the first radix-2 step reduces to
// copies.
template <bool INV>
__device__ __forceinline__ void dft8_lo(float2* v) {
    float2 e[4] = {v[0], v[2]};
    float2 o[4] = {v[1], v[3]};
    dft4_lo<INV>(e);
    dft4_lo<INV>(o);
    dft8_join<INV>(v, e, o);
}

template <int R, bool INV>
__device__ __forceinline__ void dftR(float2* v) {
    if constexpr (R == 2) dft2<INV>(v);
    else if constexpr (R == 4) dft4<INV>(v);
    else dft8<INV>(v);
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// Radix of the pass that starts at span Ns for an N-point transform: radix 8
// while possible, the remainder (2 or 4) first.
template <int N, int Ns>
constexpr int pass_radix() {
    constexpr int rem = ilog2(N / Ns);
    return (rem % 3 == 1 && Ns == 1) ? 2 : (rem % 3 == 2 && Ns == 1) ? 4 : 8;
}

// One Stockham pass over `nlines` lines of length N starting at buf + line*LS.
// Threads [0, nlines*TPL) take part in the arithmetic; every thread of the
// block must call this (it contains barriers).
template <int N, int Ns, int R, int TPL, bool INV>
__device__ __forceinline__ void stockham_pass(float2* buf, int LS, int nlines, const float2* __restrict__ tw) {
    constexpr int NB = N / R;                       // butterflies per line
    constexpr int PER = (NB + TPL - 1) / TPL;       // butterflies per thread
    const int tid = threadIdx.x;
    const int line = tid / TPL;
    const int lt = tid % TPL;
    const bool active = line < nlines;
    float2* p = buf + (size_t)(active ? line : 0) * LS;
    float2 v[PER][R];
#pragma unroll
    for (int b = 0; b < PER; ++b) {
        const int j = lt + b * TPL;
        if (active && (NB % TPL == 0 || j < NB)) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = p[j + r * NB];
            const int jm = j & (Ns - 1);
            if constexpr (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = tw[(r * jm) * (N / (Ns * R))];
                    v[b][r] = INV ? cmulc(v[b][r], w) : cmul(v[b][r], w);
                }
            }
            dftR<R, INV>(v[b]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < PER; ++b) {
        const int j = lt + b * TPL;
        if (active && (NB % TPL == 0 || j < NB)) {
            const int jm = j & (Ns - 1);
            const int base = (j - jm) * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) p[base + r * Ns] = v[b][r];
        }
    }
    __syncthreads();
}

template <int N, int Ns, int TPL, bool INV>
__device__ __forceinline__ void stockham_from(float2* buf, int LS, int nlines, const float2* __restrict__ tw) {
    if constexpr (Ns < N) {
        constexpr int R = pass_radix<N, Ns>();
        stockham_pass<N, Ns, R, TPL, INV>(buf, LS, nlines, tw);
        stockham_from<N, Ns * R, TPL, INV>(buf, LS, nlines, tw);
    }
}

// In-place N-point DFT (forward: e^{-2 pi j k n / N}; inverse: e^{+...},
// unnormalised) of `nlines` LDS lines, TPL threads per line.  The caller
// must have synchronised the block after filling the lines; on return the
// block is synchronised and the lines hold the transforms in natural order.
template <int N, int TPL, bool INV>
__device__ __forceinline__ void fft_lines(float2* buf, int LS, int nlines, const float2* __restrict__ tw) {
    stockham_from<N, 1, TPL, INV>(buf, LS, nlines, tw);
}

}  // namespace nursd
