// Plan-time host computations: the frame rule, the binning of relay samples
// for the spreading kernel, Gauss-Legendre quadrature (deconvolution tables)
// and a float64 FFT (chirp tables).  Plain C++17 without HIP, so that the
// same code also builds into a host-only test under the address and
// undefined-behaviour sanitizers.
#pragma once
#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

namespace nursd {

// Binned relay sample, one per (sample or periodic image, band) it touches.
// In centred fine-grid cells the sample sits at (ix0 + fx, iy0 + fy); its
// w x w taps are cells ix0 .. ix0 + w - 1 (x) and iy0 .. iy0 + w - 1 (y).
// Splitting the integer base from the fraction keeps the tap offsets exact
// to float precision on grids of any size.
struct SpreadEntry {
    short ix0, iy0;
    float fx, fy;
    int idx;     // relay index into P
};

// Wavefronts per spreading workgroup; each owns a contiguous range of fine
// columns of the band (chosen on the host so the waves walk similar numbers
// of samples).
constexpr int kSpreadWaves = 16;

constexpr double kPi = 3.14159265358979323846;

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n).
inline void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& wts) {
    x.resize(n);
    wts.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                x[i] = z;
                wts[i] = 2.0 / ((1.0 - z * z) * dp * dp);
                break;
            }
            x[i] = z;
            wts[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
}

// In-place iterative radix-2 FFT in float64 (plan-time tables only; the size
// is a power of two).
inline void fft64(std::vector<std::complex<double>>& a) {
    const size_t n = a.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        for (size_t i = 0; i < n; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const double ang = -2.0 * kPi * (double)k / (double)len;
                const std::complex<double> w(std::cos(ang), std::sin(ang));
                const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
    }
}

// The exponential of semicircle kernel psi(z) = exp(beta (sqrt(1 - z^2) - 1))
// on |z| < 1, zero outside.
inline double es_psi(double z, double beta) {
    double t = 1.0 - z * z;
    return t <= 0.0 ? 0.0 : std::exp(beta * (std::sqrt(t) - 1.0));
}

// Frame rule: every relay and voxel inside the period around (cx, cy) and
// every relay-voxel offset strictly inside half a period, per axis.  rxy
// holds (x, y) pairs; vlo, vhi bound the voxels.
inline bool frame_fits(int M, double dx, double dy, double cx, double cy, const std::vector<float>& rxy,
                       const double vlo[2], const double vhi[2]) {
    const double d[2] = {dx, dy}, c[2] = {cx, cy};
    for (int ax = 0; ax < 2; ++ax) {
        const double Lp = M * d[ax];
        double rmin = 1e300, rmax = -1e300;
        for (size_t i = ax; i < rxy.size(); i += 2) {
            rmin = std::min(rmin, (double)rxy[i]);
            rmax = std::max(rmax, (double)rxy[i]);
        }
        if (rmin - c[ax] < -Lp / 2 || rmax - c[ax] >= Lp / 2) return false;
        if (vlo[ax] - c[ax] < -Lp / 2 || vhi[ax] - c[ax] >= Lp / 2) return false;
        if (std::max(vhi[ax] - rmin, rmax - vlo[ax]) >= Lp / 2) return false;
    }
    return true;
}

// Relay entries of the spreading kernel for bands of BR fine rows: one entry
// per (sample or periodic image, band) it touches, sorted by band then by
// ix0, with each band's columns split between the spreading waves.
struct SpreadLists {
    int nbands = 0;
    std::vector<SpreadEntry> ent;
    std::vector<int> band_ptr;   // [nbands + 1] entry range of each band
    std::vector<int> wave_rng;   // [nbands][kSpreadWaves][4]: entry range, then column range, of each wave
};

// Fine grid of Mf x Mf cells at pitch (dx/2, dy/2) centred on (cx, cy); ES
// kernel of w taps; L relay samples at rxy (x, y pairs).  Returns false (with
// a message) when a sample lies outside the period.
inline bool bin_relays(int Mf, int w, double cx, double cy, double dx, double dy, int L,
                       const std::vector<float>& rxy, int BR, SpreadLists& sl, std::string* err) {
    const double hw = 0.5 * w;
    sl.nbands = Mf / BR;
    struct E {
        int band, ix0, iy0, l;
        float fx, fy;
    };
    std::vector<E> ents;
    ents.reserve((size_t)L * 2);
    for (int l = 0; l < L; ++l) {
        const double u = ((double)rxy[2 * l] - cx) / dx * 2.0 + Mf / 2;
        const double v = ((double)rxy[2 * l + 1] - cy) / dy * 2.0 + Mf / 2;
        if (!(u >= 0.0 && u < Mf && v >= 0.0 && v < Mf)) {
            if (err) *err = "relay sample " + std::to_string(l) + " lies outside the plan's period";
            return false;
        }
        const int ix0 = (int)std::ceil(u - hw), iy0 = (int)std::ceil(v - hw);
        const float fx = (float)(u - ix0), fy = (float)(v - iy0);
        int xs[2] = {ix0, 0}, ys[2] = {iy0, 0};
        int nxs = 1, nys = 1;
        if (ix0 < 0) xs[nxs++] = ix0 + Mf;
        if (ix0 + w - 1 >= Mf) xs[nxs++] = ix0 - Mf;
        if (iy0 < 0) ys[nys++] = iy0 + Mf;
        if (iy0 + w - 1 >= Mf) ys[nys++] = iy0 - Mf;
        for (int a = 0; a < nxs; ++a)
            for (int c = 0; c < nys; ++c) {
                const int r0 = std::max(ys[c], 0), r1 = std::min(ys[c] + w - 1, Mf - 1);
                if (r0 > r1) continue;
                for (int band = r0 / BR; band <= r1 / BR; ++band)
                    ents.push_back({band, xs[a], ys[c], l, fx, fy});
            }
    }
    std::stable_sort(ents.begin(), ents.end(), [](const E& a, const E& b) {
        return a.band != b.band ? a.band < b.band : a.ix0 < b.ix0;
    });
    sl.ent.resize(ents.size());
    sl.band_ptr.assign(sl.nbands + 1, 0);
    for (size_t i = 0; i < ents.size(); ++i) {
        sl.ent[i].ix0 = (short)ents[i].ix0;
        sl.ent[i].iy0 = (short)ents[i].iy0;
        sl.ent[i].fx = ents[i].fx;
        sl.ent[i].fy = ents[i].fy;
        sl.ent[i].idx = ents[i].l;
        sl.band_ptr[ents[i].band + 1]++;
    }
    for (int b = 0; b < sl.nbands; ++b) sl.band_ptr[b + 1] += sl.band_ptr[b];
    // Column range and entry range of each spreading wave.  The columns of a
    // band are split where the band's entries (sorted by ix0) reach equal
    // counts, so that all waves of a workgroup walk about as many samples
    // (relays usually cover only part of the period).  Taps of entry e reach
    // columns ix0 .. ix0 + w - 1, so wave columns [c_lo, c_hi) need ix0 in
    // [c_lo - w + 1, c_hi).
    constexpr int R = kSpreadWaves;                      // column ranges per band, one per wave
    sl.wave_rng.assign((size_t)sl.nbands * R * 4, 0);
    for (int b = 0; b < sl.nbands; ++b) {
        auto first = ents.begin() + sl.band_ptr[b], last = ents.begin() + sl.band_ptr[b + 1];
        const long n = last - first;
        int bound[R + 1];
        bound[0] = 0;
        bound[R] = Mf;
        for (int wv = 1; wv < R; ++wv) {
            int c = n > 0 ? (first + (n * wv) / R)->ix0 : (wv * Mf) / R;
            c = std::min(std::max(c, bound[wv - 1]), Mf);
            bound[wv] = c;
        }
        for (int wv = 0; wv < R; ++wv) {
            const int lo = bound[wv] - w + 1, hi = bound[wv + 1];
            auto a = std::lower_bound(first, last, lo, [](const E& e, int v) { return e.ix0 < v; });
            auto c = std::lower_bound(first, last, hi, [](const E& e, int v) { return e.ix0 < v; });
            int* r = &sl.wave_rng[((size_t)b * R + wv) * 4];
            r[0] = (int)(a - ents.begin());
            r[1] = (int)(c - ents.begin());
            r[2] = bound[wv];
            r[3] = bound[wv + 1];
        }
    }
    return true;
}

}  // namespace nursd
