// Host-only checks of the plan-time code in csrc/host_plan.hpp, built with
// g++ under the address and undefined-behaviour sanitizers by
// tests/test_host_sanitized.py.  Each check compares against a definition
// written out independently here (quadrature exactness, a direct DFT, the
// tap coverage of the spreading entries); the first failure exits non-zero.
#include "host_plan.hpp"

#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <tuple>

using namespace nursd;

static int g_checks = 0;
#define CHECK(cond, ...)                                         \
    do {                                                         \
        ++g_checks;                                              \
        if (!(cond)) {                                           \
            std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);                   \
            std::fprintf(stderr, "\n");                          \
            std::exit(1);                                        \
        }                                                        \
    } while (0)

// Gauss-Legendre with n nodes integrates x^k exactly on [-1, 1] for k < 2n.
static void check_gauss_legendre() {
    for (int n : {1, 2, 3, 5, 16, 128}) {
        std::vector<double> x, w;
        gauss_legendre(n, x, w);
        CHECK((int)x.size() == n && (int)w.size() == n, "sizes n=%d", n);
        for (int i = 0; i < n; ++i) CHECK(x[i] > -1.0 && x[i] < 1.0 && w[i] > 0.0, "node %d of n=%d", i, n);
        for (int i = 1; i < n; ++i) CHECK(x[i] < x[i - 1], "nodes of n=%d not strictly ordered", n);
        const int kmax = std::min(2 * n - 1, 24);
        for (int k = 0; k <= kmax; ++k) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += w[i] * std::pow(x[i], k);
            const double exact = (k % 2) ? 0.0 : 2.0 / (k + 1);
            CHECK(std::fabs(s - exact) < 1e-12, "n=%d k=%d: %.17g vs %.17g", n, k, s, exact);
        }
    }
}

// fft64 against the direct sum X[k] = sum_n x[n] e^{-2 pi j n k / N}.
static void check_fft64() {
    std::mt19937_64 rng(7);
    std::normal_distribution<double> g;
    for (size_t n : {1u, 2u, 4u, 8u, 64u, 512u, 2048u}) {
        std::vector<std::complex<double>> a(n), ref(n);
        for (auto& v : a) v = {g(rng), g(rng)};
        for (size_t k = 0; k < n; ++k) {
            std::complex<double> s = 0.0;
            for (size_t m = 0; m < n; ++m) {
                const double ang = -2.0 * kPi * (double)((m * k) % n) / (double)n;
                s += a[m] * std::complex<double>(std::cos(ang), std::sin(ang));
            }
            ref[k] = s;
        }
        fft64(a);
        double num = 0.0, den = 0.0;
        for (size_t k = 0; k < n; ++k) {
            num += std::norm(a[k] - ref[k]);
            den += std::norm(ref[k]);
        }
        CHECK(std::sqrt(num / den) < 1e-13, "fft64 n=%zu rel err %.3e", n, std::sqrt(num / den));
    }
}

static void check_es_psi() {
    for (double beta : {4.6, 16.1, 18.4}) {
        CHECK(es_psi(0.0, beta) == 1.0, "psi(0)");
        const double z = 0.999, want = std::exp(beta * (std::sqrt(1.0 - z * z) - 1.0));
        CHECK(std::fabs(es_psi(z, beta) - want) <= 1e-15 * want, "psi(0.999)");
        CHECK(es_psi(1.5, beta) == 0.0 && es_psi(-1.0001, beta) == 0.0, "psi outside");
        for (double z : {0.1, 0.5, 0.9}) {
            CHECK(es_psi(z, beta) == es_psi(-z, beta), "psi even");
            CHECK(es_psi(z, beta) > es_psi(z + 0.05, beta), "psi decreasing");
        }
    }
}

// Frame rule edges: the period is [c - Lp/2, c + Lp/2) per axis and every
// relay-voxel offset must stay strictly below Lp/2.
static void check_frame_fits() {
    const double lo[2] = {-0.1, -0.1}, hi[2] = {0.1, 0.1};
    // M = 64, d = 0.01: Lp = 0.64, half 0.32
    CHECK(frame_fits(64, 0.01, 0.01, 0.0, 0.0, {0.0f, 0.0f, 0.2f, -0.2f}, lo, hi), "inside");
    CHECK(!frame_fits(64, 0.01, 0.01, 0.0, 0.0, {0.25f, 0.0f}, lo, hi), "offset 0.35 > 0.32");
    CHECK(!frame_fits(64, 0.01, 0.01, 0.0, 0.0, {0.0f, -0.25f}, lo, hi), "offset on y");
    CHECK(frame_fits(32, 0.01, 0.01, 0.0, 0.0, {0.0f, 0.0f}, lo, hi), "a 0.32 period holds offsets of 0.1");
    const double vlo[2] = {-0.2, -0.2}, vhi[2] = {0.2, 0.2};
    CHECK(!frame_fits(32, 0.01, 0.01, 0.0, 0.0, {0.0f, 0.0f}, vlo, vhi), "voxels outside a 0.32 period");
    CHECK(frame_fits(64, 0.01, 0.01, 0.0, 0.0, {}, lo, hi), "no relays");
    // exact edges (M = 64, d = 1/64: the period is [-0.5, 0.5) per axis)
    const double elo[2] = {-0.45, 0.4}, ehi[2] = {-0.4, 0.45};
    CHECK(frame_fits(64, 1.0 / 64, 1.0 / 64, 0.0, 0.0, {-0.5f, 0.42f}, elo, ehi), "lower edge is inside");
    CHECK(!frame_fits(64, 1.0 / 64, 1.0 / 64, 0.0, 0.0, {-0.42f, 0.5f}, elo, ehi), "upper edge is outside");
}

// Brute-force coverage of the spreading entries: every (relay, tap) cell of
// the w x w footprint, wrapped onto the period, must be reached by exactly
// one entry of the band holding that row, and the waves' entry ranges must
// hold every entry whose taps reach their columns.
static void check_bins(int Mf, int w, int BR, const std::vector<float>& rxy, double cx, double cy, double dx,
                       double dy) {
    const int L = (int)rxy.size() / 2;
    SpreadLists sl;
    std::string err;
    CHECK(bin_relays(Mf, w, cx, cy, dx, dy, L, rxy, BR, sl, &err), "bin_relays failed: %s", err.c_str());
    CHECK(sl.nbands == Mf / BR, "nbands");
    CHECK((int)sl.band_ptr.size() == sl.nbands + 1 && sl.band_ptr[0] == 0 &&
              sl.band_ptr[sl.nbands] == (int)sl.ent.size(), "band_ptr ends");
    std::multiset<std::tuple<int, int, int>> got, want;
    for (int b = 0; b < sl.nbands; ++b) {
        CHECK(sl.band_ptr[b] <= sl.band_ptr[b + 1], "band_ptr monotone");
        for (int i = sl.band_ptr[b]; i < sl.band_ptr[b + 1]; ++i) {
            const SpreadEntry& e = sl.ent[i];
            if (i > sl.band_ptr[b]) CHECK(sl.ent[i - 1].ix0 <= e.ix0, "band %d not sorted by ix0", b);
            CHECK(e.idx >= 0 && e.idx < L, "entry relay index");
            bool any = false;
            for (int ty = 0; ty < w; ++ty)
                for (int tx = 0; tx < w; ++tx) {
                    const int x = e.ix0 + tx, y = e.iy0 + ty;
                    if (x < 0 || x >= Mf || y < 0 || y >= Mf || y / BR != b) continue;
                    got.insert({e.idx, x, y});
                    any = true;
                }
            CHECK(any, "entry %d of band %d reaches no cell of its band", i, b);
        }
    }
    for (int l = 0; l < L; ++l) {
        const double u = ((double)rxy[2 * l] - cx) / dx * 2.0 + Mf / 2;
        const double v = ((double)rxy[2 * l + 1] - cy) / dy * 2.0 + Mf / 2;
        const int ix0 = (int)std::ceil(u - 0.5 * w), iy0 = (int)std::ceil(v - 0.5 * w);
        for (int ty = 0; ty < w; ++ty)
            for (int tx = 0; tx < w; ++tx)
                want.insert({l, ((ix0 + tx) % Mf + Mf) % Mf, ((iy0 + ty) % Mf + Mf) % Mf});
    }
    CHECK(got == want, "tap coverage differs (%zu cells reached, %zu wanted)", got.size(), want.size());
    // wave ranges: contiguous column split of [0, Mf); entry ranges hold
    // every entry of the band whose taps reach the wave's columns
    const int R = kSpreadWaves;
    CHECK((int)sl.wave_rng.size() == sl.nbands * R * 4, "wave_rng size");
    for (int b = 0; b < sl.nbands; ++b) {
        int prev_hi = 0;
        for (int wv = 0; wv < R; ++wv) {
            const int* r = &sl.wave_rng[((size_t)b * R + wv) * 4];
            CHECK(r[2] == prev_hi && r[2] <= r[3], "band %d wave %d column range", b, wv);
            prev_hi = r[3];
            CHECK(sl.band_ptr[b] <= r[0] && r[0] <= r[1] && r[1] <= sl.band_ptr[b + 1], "band %d wave %d entries", b, wv);
            for (int i = sl.band_ptr[b]; i < sl.band_ptr[b + 1]; ++i) {
                const int x0 = sl.ent[i].ix0;
                const bool reaches = x0 <= r[3] - 1 && x0 + w - 1 >= r[2] && r[2] < r[3];
                if (reaches) CHECK(i >= r[0] && i < r[1], "band %d wave %d misses entry %d", b, wv, i);
            }
        }
        CHECK(prev_hi == Mf, "band %d columns end at %d", b, prev_hi);
    }
}

static void check_bin_relays() {
    std::mt19937_64 rng(11);
    for (int Mf : {128, 256}) {
        const double dx = 0.02, dy = 0.025, cx = 0.1, cy = -0.05;
        const double hx = Mf * dx / 4, hy = Mf * dy / 4;   // half period (fine pitch is d / 2)
        std::uniform_real_distribution<double> ux(cx - 0.999 * hx, cx + 0.999 * hx), uy(cy - 0.999 * hy, cy + 0.999 * hy);
        for (int w : {2, 5, 7, 8})
            for (int BR : {1, 2, 4, 8, 16}) {
                // random relays, some duplicated
                std::vector<float> rxy;
                for (int l = 0; l < 300; ++l) {
                    rxy.push_back((float)ux(rng));
                    rxy.push_back((float)uy(rng));
                }
                rxy.push_back(rxy[0]);
                rxy.push_back(rxy[1]);
                check_bins(Mf, w, BR, rxy, cx, cy, dx, dy);
                // relays on the edges of the period (periodic images in x, y
                // and both), at the centre, and none at all
                const double in = 0.99999;       // float positions a hair inside the period
                std::vector<float> edge = {(float)(cx - in * hx), (float)(cy - in * hy), (float)(cx + in * hx),
                                           (float)(cy + in * hy), (float)(cx - in * hx), (float)(cy + in * hy),
                                           (float)cx, (float)cy};
                check_bins(Mf, w, BR, edge, cx, cy, dx, dy);
                check_bins(Mf, w, BR, {}, cx, cy, dx, dy);
            }
        // a relay outside the period is refused with a message
        SpreadLists sl;
        std::string err;
        const std::vector<float> out = {(float)(cx + 1.01 * hx), (float)cy};
        CHECK(!bin_relays(Mf, 7, cx, cy, dx, dy, 1, out, 8, sl, &err) && !err.empty(), "outside relay accepted");
    }
}

int main() {
    check_gauss_legendre();
    check_fft64();
    check_es_psi();
    check_frame_fits();
    check_bin_relays();
    std::printf("host plan checks ok (%d)\n", g_checks);
    return 0;
}
