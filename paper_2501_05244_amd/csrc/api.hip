// Host side of the C ABI declared in include/nursd.h: plan creation (frame
// rule, frequency bins, device tables, binning of relay samples for the
// spreading kernel, workspace layout) and the launch sequences of the
// forward operator.
#include "nursd.h"
#include "kernels.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>
#include <tuple>
#include <string>
#include <vector>

using namespace nursd;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(NURSD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define NURSD_GUARD(call)                                                   \
    do {                                                                    \
        try {                                                               \
            return call;                                                    \
        } catch (const std::exception& ex_) {                               \
            return fail(NURSD_ERR_HIP, std::string("host exception: ") + ex_.what()); \
        } catch (...) {                                                     \
            return fail(NURSD_ERR_HIP, "host exception");                   \
        }                                                                   \
    } while (0)

constexpr int kSupportedM[] = {64, 128, 256, 512, 1024};

// Spreading tile of the plans' own launches (spread_var(band rows,
// frequencies per workgroup)), for 3D (depth-mode) plans and others: one
// fine row of 8 frequencies measured fastest (with 32 frequencies per
// launch: SPAD spreading 0.77 ms against 0.86 for one row of 16, 0.90 for
// 2 x 8 and 1.03 for 4 x 4; 3D stage-1 spreading 12.1 ms against 13.1,
// 14.3 and 16.4): every lane of a step works on one copy of a tap row, and
// two workgroups share a CU.  Sizes whose tile does not fit LDS fall back
// to 8 x 2 (or 8 x 1).
#ifndef NURSD_PLAN_SPREAD_VAR
#define NURSD_PLAN_SPREAD_VAR 108
#endif
#ifndef NURSD_PLAN3D_SPREAD_VAR
#define NURSD_PLAN3D_SPREAD_VAR 108
#endif
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

struct nursd_plan {
    // wavelet
    int F = 0, T = 0, coherent = 1;
    int kernel_inv_r = 1;           // G = e^{jkr}/r (1) or e^{jkr} (0)
    double lambda_c = 0, sigma_rel = 0.2, dt = 0, t0 = 0;
    std::vector<int> bins;
    std::vector<double> freqs;
    // geometry
    int mode = NURSD_MODE_GRID;
    double x0 = 0, y0 = 0, vdx = 0, vdy = 0;
    int nx = 0, ny = 0, nz = 0;
    std::vector<double> z, alpha;
    std::vector<int> plane_ptr;
    const float* voxel_xy_dev = nullptr;
    double zref = 0;
    double xp[3] = {0, 0, 0};
    int L = 0;
    // frame
    int M = 0, Mf = 0;
    double dx = 0, dy = 0, cx = 0, cy = 0;
    int w = 7;
    double beta = 0;
    double pad = 2.0;
    int q = 1;                      // internal grid pitch = voxel pitch / q
    double vlo[2] = {0, 0}, vhi[2] = {0, 0};   // voxel bounds (frame rule of set_points)
    float* d_w = nullptr;           // [L] per-sample weights or NULL
    // chunking
    int FC = 8, ZC = 16, FCn = 16;
    int BS = 0;
    // device tables
    std::vector<void*> owned;
    float2* tw_all = nullptr;
    size_t tw_off[kMaxLog] = {};
    int* d_bins = nullptr;
    float2* d_wt = nullptr;
    float2* d_tb = nullptr;
    double* d_f = nullptr;
    double* d_z = nullptr;
    double* d_px = nullptr;   // per-plane pitch (SRSD)
    double* d_py = nullptr;
    double* d_alpha = nullptr;
    float2* d_hhat = nullptr; // [Z][2M] chirp spectra (SRSD)
    float2* d_chirp = nullptr; // [Z][M] chirps e^{-j pi alpha m^2 / M} (SRSD)
    float* d_relay = nullptr;     // [L][2] plan-owned copy of the relay positions
    int relay_row_lo = 0, relay_row_hi = -1;
    int FC3 = 4;                  // frequencies per adjoint type-2 chunk
    int* d_plane_ptr = nullptr;   // POINTS
    int* d_row_lo = nullptr;
    int* d_row_hi = nullptr;
    int* d_plane_band = nullptr;  // interpolation entries of voxel lists (see Type2Args)
    int* d_lband_ptr = nullptr;
    int* d_ent_vox = nullptr;
    int* d_vox_ent = nullptr;
    int n_lent = 0;
    int max_vox = 0;
    float* d_decx = nullptr;
    float* d_decy = nullptr;
    SpreadEntry* d_ent = nullptr;
    int* d_band_ptr = nullptr;
    int* d_wave_rng = nullptr;
    int nbands = 0, n_ent = 0;
    int spread_var = 0;           // spreading tile of the plan's own launches (spread_var)
    std::vector<float> h_relay;   // host copy of the binned relay positions [L][2]
    // per-kernel event timing
    uint32_t prof_mask = 0;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<int> ev_stage;
    // workspace layout
    size_t off_P = 0, off_T1 = 0, off_U = 0, off_Bt = 0, off_Yt = 0, off_V = 0, ws_bytes = 0;
    size_t off_Tg = 0, off_u = 0, off_S1 = 0, off_T2 = 0, off_PT = 0, off_T3 = 0, off_G3 = 0;
    // 3D NURSD: intermediate plane, depth grid, depth weights per relay
    double z_mid = 0, dz3 = 0;
    int Mz3 = 0, FZ3 = 1;           // depth size; frequencies per stage-1 chunk
    float2* d_W3 = nullptr;         // [Mz3][L]
    double* d_zk3 = nullptr;        // [Mz3] depth offsets |p dz3| of the kernel planes
    size_t off_Q3 = 0, off_Ut3 = 0;

    ~nursd_plan() {
        for (void* p : owned) (void)hipFree(p);
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    }
    bool has_lists() const { return mode == NURSD_MODE_POINTS || mode == NURSD_MODE_SRSD_POINTS; }
    bool scaled() const { return mode == NURSD_MODE_SRSD || mode == NURSD_MODE_SRSD_POINTS; }
    const float2* tw(int n) const { return tw_all + tw_off[__builtin_ctz((unsigned)n)]; }
    int nvox() const {
        return has_lists() ? (plane_ptr.empty() ? 0 : plane_ptr.back()) : nx * ny * nz;
    }
};

namespace {

// Launch `call` (a hipError_t expression) for `stage`, bracketed by events
// when that stage is being profiled.
int timed(nursd_plan* p, int stage, hipStream_t s, hipError_t (*fn)(const void*, hipStream_t), const void* args) {
    const bool on = (p->prof_mask >> stage) & 1u;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (on) {
        while (p->ev_pool.size() < p->ev_used + 2) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            p->ev_pool.push_back(e);
        }
        e0 = p->ev_pool[p->ev_used];
        e1 = p->ev_pool[p->ev_used + 1];
        HIP_TRY(hipEventRecord(e0, s));
    }
    HIP_TRY(fn(args, s));
    if (on) {
        HIP_TRY(hipEventRecord(e1, s));
        p->ev_used += 2;
        p->ev_stage.push_back(stage);
    }
    return NURSD_OK;
}

template <typename A, hipError_t (*L)(const A&, hipStream_t)>
hipError_t thunk(const void* a, hipStream_t s) {
    return L(*static_cast<const A*>(a), s);
}

#define LAUNCH(p, stage, Args, launcher, args, s)                                   \
    do {                                                                             \
        int rc_ = timed(p, stage, s, &thunk<Args, launcher>, &(args));               \
        if (rc_) return rc_;                                                         \
    } while (0)

template <typename T>
int upload(nursd_plan* p, const std::vector<T>& v, T** out) {
    *out = nullptr;
    if (v.empty()) return NURSD_OK;
    void* d = nullptr;
    HIP_TRY(hipMalloc(&d, v.size() * sizeof(T)));
    p->owned.push_back(d);
    HIP_TRY(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    *out = static_cast<T*>(d);
    return NURSD_OK;
}

// Binning of the relay samples for bands of BR fine rows (host_plan.hpp).
int bin_relays(const nursd_plan* p, const std::vector<float>& rxy, int BR, SpreadLists& sl) {
    std::string err;
    if (!nursd::bin_relays(p->Mf, p->w, p->cx, p->cy, p->dx, p->dy, p->L, rxy, BR, sl, &err))
        return fail(NURSD_ERR_GEOMETRY, err);
    return NURSD_OK;
}

int build_spread_lists(nursd_plan* p, const std::vector<float>& rxy) {
    const int Mf = p->Mf, w = p->w;
    const double hw = 0.5 * w;
    SpreadLists sl;
    if (int rc = bin_relays(p, rxy, spread_var_rows(p->spread_var, Mf), sl)) return rc;
    p->nbands = sl.nbands;
    p->n_ent = (int)sl.ent.size();
    p->h_relay = rxy;
    const std::vector<SpreadEntry>& out = sl.ent;
    const std::vector<int>& ptr = sl.band_ptr;
    const std::vector<int>& rng = sl.wave_rng;
    if (p->d_ent) {
        // replace previous lists
        for (auto it = p->owned.begin(); it != p->owned.end();) {
            if (*it == (void*)p->d_ent || *it == (void*)p->d_band_ptr || *it == (void*)p->d_wave_rng) {
                (void)hipFree(*it);
                it = p->owned.erase(it);
            } else {
                ++it;
            }
        }
        p->d_ent = nullptr;
        p->d_band_ptr = nullptr;
        p->d_wave_rng = nullptr;
    }
    // relay fine rows reached by interpolation (adjoint type-2 at relay points)
    {
        int lo = 1 << 30, hi = -(1 << 30);
        for (int l = 0; l < p->L; ++l) {
            const double v = ((double)rxy[2 * l + 1] - p->cy) / p->dy * 2.0 + Mf / 2;
            const int iy0 = (int)std::ceil(v - hw);
            lo = std::min(lo, iy0);
            hi = std::max(hi, iy0 + w - 1);
        }
        if (hi - lo + 1 >= Mf) {
            lo = 0;
            hi = Mf - 1;
        }
        p->relay_row_lo = lo;
        p->relay_row_hi = hi;
    }
    int rc;
    if (!p->d_relay) {
        void* d = nullptr;
        HIP_TRY(hipMalloc(&d, (size_t)p->L * 2 * sizeof(float)));
        p->owned.push_back(d);
        p->d_relay = static_cast<float*>(d);
    }
    HIP_TRY(hipMemcpy(p->d_relay, rxy.data(), (size_t)p->L * 2 * sizeof(float), hipMemcpyHostToDevice));
    if ((rc = upload(p, out, &p->d_ent))) return rc;
    if ((rc = upload(p, rng, &p->d_wave_rng))) return rc;
    return upload(p, ptr, &p->d_band_ptr);
}

int read_points(const float* dev, size_t n2, std::vector<float>& host, hipStream_t s) {
    host.resize(n2);
    HIP_TRY(hipMemcpyAsync(host.data(), dev, n2 * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return NURSD_OK;
}

void layout_workspace(nursd_plan* p) {
    size_t o = 0;
    const size_t c8 = sizeof(float2);
    p->off_P = o;
    o = align_up(o + (size_t)p->F * p->L * c8);
    p->off_T1 = o;
    o = align_up(o + (size_t)p->FCn * p->M * p->Mf * c8);
    p->off_U = o;
    o = align_up(o + (size_t)p->F * p->M * p->M * c8);
    const size_t planes = (size_t)p->FC * p->ZC;
    const size_t kplanes = std::max(planes, (size_t)p->FZ3 * p->Mz3);   // kernel rows: also the 3D stage
    p->off_Bt = o;
    o = align_up(o + kplanes * (p->M / 2 + 1) * p->BS * c8);
    p->off_Yt = o;
    o = align_up(o + planes * p->ny * p->M * c8);
    if (p->has_lists()) {
        p->off_T2 = o;
        o = align_up(o + planes * p->M * p->Mf * c8);
        p->off_PT = o;
        o = align_up(o + (size_t)p->FC * std::max(p->n_lent, 1) * c8);
    }
    p->off_V = o;
    o = align_up(o + (size_t)p->nvox() * c8);
    if (p->mode == NURSD_MODE_GRID && p->coherent) {
        p->off_T3 = o;
        o = align_up(o + (size_t)p->FC3 * 3 * p->M * p->Mf * c8);
        p->off_G3 = o;
        o = align_up(o + (size_t)p->FC3 * 3 * p->Mf * p->Mf * c8);
    }
    if (p->mode == NURSD_MODE_GRID3D) {
        p->off_Q3 = o;
        o = align_up(o + (size_t)p->Mz3 * p->FZ3 * p->L * c8);
        p->off_Ut3 = o;
        o = align_up(o + (size_t)p->Mz3 * p->FZ3 * p->M * p->M * c8);
    }
    if (p->scaled()) {
        p->off_Tg = o;
        o = align_up(o + (size_t)p->F * p->M * p->nx * c8);
        p->off_u = o;
        o = align_up(o + (size_t)p->F * p->nx * p->nx * c8);
        p->off_S1 = o;
        o = align_up(o + planes * p->M * p->nx * c8);
    }
    p->ws_bytes = o;
}

int check_ws(const nursd_plan* p, void* ws, size_t bytes) {
    if (!ws) return fail(NURSD_ERR_WORKSPACE, "workspace pointer is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(NURSD_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (bytes < p->ws_bytes)
        return fail(NURSD_ERR_WORKSPACE, "workspace too small: need " + std::to_string(p->ws_bytes) + " bytes");
    return NURSD_OK;
}

// Copies the CSR plane pointers and reads the voxel positions to the host.
int read_voxel_lists(nursd_plan* p, const nursd_geometry* geo, std::vector<float>& vxy, hipStream_t s) {
    p->plane_ptr.assign(geo->plane_ptr, geo->plane_ptr + p->nz + 1);
    p->voxel_xy_dev = geo->voxel_xy_dev;
    const int V = p->plane_ptr.back();
    for (int i = 0; i < p->nz; ++i)
        if (p->plane_ptr[i + 1] < p->plane_ptr[i]) return fail(NURSD_ERR_ARG, "plane_ptr must be non-decreasing");
    if (p->plane_ptr[0] != 0 || V < 1) return fail(NURSD_ERR_ARG, "plane_ptr must start at 0 and list voxels");
    return read_points(geo->voxel_xy_dev, (size_t)V * 2, vxy, s);
}

bool even_bins(const nursd_plan* p) {
    for (int b = 2; b < p->F; ++b)
        if (p->bins[b] - p->bins[b - 1] != p->bins[1] - p->bins[0]) return false;
    return true;
}

ChunkGeom chunk_geom(const nursd_plan* p, int b0, int nb, int z0, int nzc) {
    ChunkGeom g;
    g.b0 = b0;
    g.nb = nb;
    g.z0 = z0;
    g.nzc = nzc;
    g.f = p->d_f;
    g.z = p->d_z;
    g.pitch_x = p->d_px;
    g.pitch_y = p->d_py;
    g.dx = p->dx;
    g.dy = p->dy;
    // Evenly spaced bins let the kernels advance phases by a per-point step
    // factor from one frequency to the next instead of evaluating each.
    g.uni = 1;
    g.df = 0.0;
    if (nb > 1) {
        const int step = p->bins[b0 + 1] - p->bins[b0];
        for (int b = b0 + 1; b < b0 + nb; ++b)
            if (p->bins[b] - p->bins[b - 1] != step) g.uni = 0;
        g.df = g.uni ? p->freqs[b0 + 1] - p->freqs[b0] : 0.0;
    }
    return g;
}

// Argument blocks of the three propagation passes.
P1Args kernel_args(const nursd_plan* p, const ChunkGeom& g, float2* Bt) {
    P1Args a{g, Bt, p->M, p->BS, p->tw(p->M)};
    a.plain = p->kernel_inv_r ? 0 : 1;
    return a;
}

P2Args cols_args(const nursd_plan* p, const ChunkGeom& g, const float2* Bt, const float2* U, float2* Yt) {
    P2Args a{g, Bt, U, Yt, p->M, p->BS, p->ny, p->tw(p->M)};
    a.q = p->q;
    return a;
}

// Type-1 NUFFT of n rows of P ([n][L], n = F by default) -> U [n][M][M].
int run_spectrum(nursd_plan* p, const float2* P, float2* U, char* ws, hipStream_t s, int n = -1) {
    if (n < 0) n = p->F;
    for (int b0 = 0; b0 < n; b0 += p->FCn) {
        const int nb = std::min(p->FCn, n - b0);
        SpreadArgs sa{};
        sa.var = p->spread_var;
        sa.P = P;
        sa.wts = p->d_w;
        sa.ent = p->d_ent;
        sa.band_ptr = p->d_band_ptr;
        sa.wave_rng = p->d_wave_rng;
        sa.T1 = reinterpret_cast<float2*>(ws + p->off_T1);
        sa.decx = p->d_decx;
        sa.tw = p->tw(p->Mf);
        sa.M = p->M;
        sa.Mf = p->Mf;
        sa.L = p->L;
        sa.w = p->w;
        sa.beta = (float)p->beta;
        sa.half_w = 0.5f * p->w;
        sa.b0 = b0;
        sa.nb = nb;
        LAUNCH(p, NURSD_STAGE_SPREAD, SpreadArgs, launch_spread_xfft, sa, s);
        FineYArgs fa{};
        fa.T1 = sa.T1;
        fa.U = U;
        fa.decy = p->d_decy;
        fa.tw = p->tw(p->Mf);
        fa.M = p->M;
        fa.Mf = p->Mf;
        fa.b0 = b0;
        fa.nb = nb;
        fa.br = spread_var_rows(p->spread_var, p->Mf);
        LAUNCH(p, NURSD_STAGE_FINE_Y, FineYArgs, launch_fine_y, fa, s);
    }
    return NURSD_OK;
}

P3Args rows_args(const nursd_plan* p, const ChunkGeom& g, const float2* Yt, float2* V, float* I, int b0, int nb);

int run_grid_propagation(nursd_plan* p, const float2* U, float2* V, float* I, char* ws, hipStream_t s) {
    float2* Bt = reinterpret_cast<float2*>(ws + p->off_Bt);
    float2* Yt = reinterpret_cast<float2*>(ws + p->off_Yt);
    for (int b0 = 0; b0 < p->F; b0 += p->FC) {
        const int nb = std::min(p->FC, p->F - b0);
        for (int z0 = 0; z0 < p->nz; z0 += p->ZC) {
            const int nzc = std::min(p->ZC, p->nz - z0);
            const ChunkGeom g = chunk_geom(p, b0, nb, z0, nzc);
            P1Args a1 = kernel_args(p, g, Bt);
            LAUNCH(p, NURSD_STAGE_KERNEL_ROWS, P1Args, launch_kernel_rows, a1, s);
            P2Args a2 = cols_args(p, g, Bt, U, Yt);
            LAUNCH(p, NURSD_STAGE_PROPAGATE_COLS, P2Args, launch_propagate_cols, a2, s);
            P3Args a3 = rows_args(p, g, Yt, V, I, b0, nb);
            LAUNCH(p, NURSD_STAGE_PROPAGATE_ROWS, P3Args, launch_propagate_rows, a3, s);
        }
    }
    return NURSD_OK;
}

P3Args rows_args(const nursd_plan* p, const ChunkGeom& g, const float2* Yt, float2* V, float* I, int b0, int nb) {
    P3Args a3{};
    a3.g = g;
    a3.Yt = Yt;
    a3.V = V;
    a3.I = I;
    a3.M = p->M;
    a3.nx = p->nx;
    a3.ny = p->ny;
    a3.xc = p->cx;
    a3.yc = p->cy;
    a3.xp0 = p->xp[0];
    a3.xp1 = p->xp[1];
    a3.xp2 = p->xp[2];
    a3.first = b0 == 0;
    a3.last = b0 + nb >= p->F;
    a3.coherent = p->coherent;
    a3.tw = p->tw(p->M);
    a3.q = p->q;
    return a3;
}

int run_srsd(nursd_plan* p, const float2* U, float2* V, float* I, char* ws, hipStream_t s) {
    float2* Bt = reinterpret_cast<float2*>(ws + p->off_Bt);
    float2* Yt = reinterpret_cast<float2*>(ws + p->off_Yt);
    float2* u = reinterpret_cast<float2*>(ws + p->off_u);
    RelayGridArgs ra{};
    ra.U = U;
    ra.Tg = reinterpret_cast<float2*>(ws + p->off_Tg);
    ra.u = u;
    ra.M = p->M;
    ra.N = p->nx;
    ra.b0 = 0;
    ra.nb = p->F;
    ra.tw_m = p->tw(p->M);
    LAUNCH(p, NURSD_STAGE_RELAY_GRID, RelayGridArgs, launch_relay_grid, ra, s);
    for (int b0 = 0; b0 < p->F; b0 += p->FC) {
        const int nb = std::min(p->FC, p->F - b0);
        for (int z0 = 0; z0 < p->nz; z0 += p->ZC) {
            const int nzc = std::min(p->ZC, p->nz - z0);
            const ChunkGeom g = chunk_geom(p, b0, nb, z0, nzc);
            P1Args a1 = kernel_args(p, g, Bt);
            LAUNCH(p, NURSD_STAGE_KERNEL_ROWS, P1Args, launch_kernel_rows, a1, s);
            ChirpArgs ca{};
            ca.g = g;
            ca.u = u;
            ca.S1t = reinterpret_cast<float2*>(ws + p->off_S1);
            ca.Bt = Bt;
            ca.Yt = Yt;
            ca.M = p->M;
            ca.N = p->nx;
            ca.BS = p->BS;
            ca.ny = p->ny;
            ca.alpha = p->d_alpha;
            ca.hhat = p->d_hhat;
            ca.chirp = p->d_chirp;
            ca.tw_m = p->tw(p->M);
            ca.tw_lb = p->tw(2 * p->M);
            LAUNCH(p, NURSD_STAGE_CHIRP_ROWS, ChirpArgs, launch_chirp_rows, ca, s);
            LAUNCH(p, NURSD_STAGE_PROPAGATE_COLS, ChirpArgs, launch_chirp_cols, ca, s);
            P3Args a3 = rows_args(p, g, Yt, V, I, b0, nb);
            LAUNCH(p, NURSD_STAGE_PROPAGATE_ROWS, P3Args, launch_propagate_rows, a3, s);
        }
    }
    return NURSD_OK;
}

Type2Args type2_args(const nursd_plan* p, const ChunkGeom& g, const float2* Bt, const float2* U, float2* V, float* I,
                     char* ws, int b0, int nb);

int run_points(nursd_plan* p, const float2* U, float2* V, float* I, char* ws, hipStream_t s) {
    float2* Bt = reinterpret_cast<float2*>(ws + p->off_Bt);
    for (int b0 = 0; b0 < p->F; b0 += p->FC) {
        const int nb = std::min(p->FC, p->F - b0);
        for (int z0 = 0; z0 < p->nz; z0 += p->ZC) {
            const int nzc = std::min(p->ZC, p->nz - z0);
            const ChunkGeom g = chunk_geom(p, b0, nb, z0, nzc);
            P1Args a1 = kernel_args(p, g, Bt);
            LAUNCH(p, NURSD_STAGE_KERNEL_ROWS, P1Args, launch_kernel_rows, a1, s);
            Type2Args t = type2_args(p, g, Bt, U, V, I, ws, b0, nb);
            LAUNCH(p, NURSD_STAGE_TYPE2, Type2Args, launch_type2, t, s);
        }
    }
    return NURSD_OK;
}

Type2Args type2_args(const nursd_plan* p, const ChunkGeom& g, const float2* Bt, const float2* U, float2* V, float* I,
                     char* ws, int b0, int nb) {
    Type2Args t{};
    t.g = g;
    t.Bt = Bt;
    t.U = U;
    t.T2 = reinterpret_cast<float2*>(ws + p->off_T2);
    t.part = reinterpret_cast<float2*>(ws + p->off_PT);
    t.n_lent = p->n_lent;
    t.plane_band = p->d_plane_band;
    t.band_ptr = p->d_lband_ptr;
    t.ent_vox = p->d_ent_vox;
    t.vox_ent = p->d_vox_ent;
    t.V = V;
    t.I = I;
    t.dec = p->d_decy;
    t.tw_m = p->tw(p->M);
    t.tw_f = p->tw(p->Mf);
    t.M = p->M;
    t.Mf = p->Mf;
    t.BS = p->BS;
    t.w = p->w;
    t.beta = (float)p->beta;
    t.cx = p->cx;
    t.cy = p->cy;
    t.xp0 = p->xp[0];
    t.xp1 = p->xp[1];
    t.xp2 = p->xp[2];
    t.plane_ptr = p->d_plane_ptr;
    t.voxel_xy = p->voxel_xy_dev;
    t.row_lo = p->d_row_lo;
    t.row_hi = p->d_row_hi;
    t.max_vox = p->max_vox;
    t.first = b0 == 0;
    t.last = b0 + nb >= p->F;
    t.coherent = p->coherent;
    return t;
}

// Scaled RSD evaluated at per-plane voxel lists (eq. NURSD2_SRSD): relay
// grid, kernel rows at pitch d/alpha, Bluestein rows, then per column the
// scaled spectrum times the kernel spectrum handed to the type-2 steps.
int run_srsd_points(nursd_plan* p, const float2* U, float2* V, float* I, char* ws, hipStream_t s) {
    float2* Bt = reinterpret_cast<float2*>(ws + p->off_Bt);
    float2* u = reinterpret_cast<float2*>(ws + p->off_u);
    RelayGridArgs ra{};
    ra.U = U;
    ra.Tg = reinterpret_cast<float2*>(ws + p->off_Tg);
    ra.u = u;
    ra.M = p->M;
    ra.N = p->nx;
    ra.b0 = 0;
    ra.nb = p->F;
    ra.tw_m = p->tw(p->M);
    LAUNCH(p, NURSD_STAGE_RELAY_GRID, RelayGridArgs, launch_relay_grid, ra, s);
    for (int b0 = 0; b0 < p->F; b0 += p->FC) {
        const int nb = std::min(p->FC, p->F - b0);
        for (int z0 = 0; z0 < p->nz; z0 += p->ZC) {
            const int nzc = std::min(p->ZC, p->nz - z0);
            const ChunkGeom g = chunk_geom(p, b0, nb, z0, nzc);
            P1Args a1 = kernel_args(p, g, Bt);
            LAUNCH(p, NURSD_STAGE_KERNEL_ROWS, P1Args, launch_kernel_rows, a1, s);
            ChirpArgs ca{};
            ca.g = g;
            ca.u = u;
            ca.S1t = reinterpret_cast<float2*>(ws + p->off_S1);
            ca.Bt = Bt;
            ca.M = p->M;
            ca.N = p->nx;
            ca.BS = p->BS;
            ca.ny = p->ny;
            ca.alpha = p->d_alpha;
            ca.hhat = p->d_hhat;
            ca.chirp = p->d_chirp;
            ca.tw_m = p->tw(p->M);
            ca.tw_lb = p->tw(2 * p->M);
            ca.T2 = reinterpret_cast<float2*>(ws + p->off_T2);
            ca.dec = p->d_decy;
            ca.row_lo = p->d_row_lo;
            ca.row_hi = p->d_row_hi;
            LAUNCH(p, NURSD_STAGE_CHIRP_ROWS, ChirpArgs, launch_chirp_rows, ca, s);
            LAUNCH(p, NURSD_STAGE_PROPAGATE_COLS, ChirpArgs, launch_chirp_type2_cols, ca, s);
            Type2Args t = type2_args(p, g, Bt, U, V, I, ws, b0, nb);
            LAUNCH(p, NURSD_STAGE_TYPE2, Type2Args, launch_type2_fine, t, s);
        }
    }
    return NURSD_OK;
}

// 3D NURSD stage 1: the spectrum U0 of the field on the intermediate plane.
int run_stage1_3d(nursd_plan* p, const float2* P, float2* U0, char* ws, hipStream_t s) {
    float2* Q = reinterpret_cast<float2*>(ws + p->off_Q3);
    float2* Ut = reinterpret_cast<float2*>(ws + p->off_Ut3);
    float2* Bt = reinterpret_cast<float2*>(ws + p->off_Bt);
    for (int b0 = 0; b0 < p->F; b0 += p->FZ3) {
        const int nb = std::min(p->FZ3, p->F - b0);
        ModulateArgs ma{P, p->d_W3, Q, p->L, p->Mz3, b0, nb};
        LAUNCH(p, NURSD_STAGE_NURSD3D, ModulateArgs, launch_modulate, ma, s);
        int rc = run_spectrum(p, Q, Ut, ws, s, p->Mz3 * nb);
        if (rc) return rc;
        ChunkGeom g = chunk_geom(p, b0, nb, 0, p->Mz3);
        g.z = p->d_zk3;
        g.pitch_x = g.pitch_y = nullptr;
        P1Args a1 = kernel_args(p, g, Bt);
        a1.plain = 1;                      // the 3D-RSD kernel e^{+jkr} (no 1/r)
        LAUNCH(p, NURSD_STAGE_KERNEL_ROWS, P1Args, launch_kernel_rows, a1, s);
        Stage1Args sa{g, Bt, Ut, U0, p->M, p->BS, p->Mz3, p->tw(p->M)};
        LAUNCH(p, NURSD_STAGE_NURSD3D, Stage1Args, launch_stage1_reduce, sa, s);
    }
    return NURSD_OK;
}

int forward_from_P(nursd_plan* p, const float2* P, void* vol, float* I, char* ws, hipStream_t s) {
    float2* U = reinterpret_cast<float2*>(ws + p->off_U);
    int rc = p->mode == NURSD_MODE_GRID3D ? run_stage1_3d(p, P, U, ws, s) : run_spectrum(p, P, U, ws, s);
    if (rc) return rc;
    float2* V = vol ? static_cast<float2*>(vol) : reinterpret_cast<float2*>(ws + p->off_V);
    if (!p->coherent) V = nullptr;
    if (p->mode == NURSD_MODE_SRSD) return run_srsd(p, U, V, I, ws, s);
    if (p->mode == NURSD_MODE_POINTS) return run_points(p, U, V, I, ws, s);
    if (p->mode == NURSD_MODE_SRSD_POINTS) return run_srsd_points(p, U, V, I, ws, s);
    return run_grid_propagation(p, U, V, I, ws, s);
}

}  // namespace


// ============================================================================
// Batched serving: many GRID plans in one captured graph of grouped
// persistent launches.
// ============================================================================
__global__ void k_zero_counters(int* c, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0;
}

namespace nursd {
hipError_t launch_zero_counters(int* c, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_counters, dim3((n + 255) / 256), dim3(256), 0, s, c, n);
    return hipGetLastError();
}
}  // namespace nursd

enum { BK_PHASOR = 0, BK_SPREAD, BK_FINEY, BK_P1, BK_P2, BK_P3, BK_SERIAL, BK_KTAB, BK_MULTI };

// One configuration of the batched launch sequence.
struct BatchConfig {
    int rounds = 4;            // propagation rounds R of the grouped scenes
    int sched = kQueue;        // grouped-launch schedule (kQueue, kStatic, kFlat)
    int serial_min_m = 512;    // scenes with M >= this are propagated chunk by chunk
    int share = 1;             // kernel spectra shared by the scenes of a kernel class
};

int config_code(const BatchConfig& c) {
    return c.rounds + 1000 * c.sched + 10000 * (c.serial_min_m == 256 ? 1 : c.serial_min_m == 512 ? 2 : 0) +
           100000 * c.share;
}

// Scenes whose kernels G(m dx, n dy, z) = e^{+j 2 pi f r / c} / r agree in
// transform size, pitch and amplitude form form a kernel class: the kernel
// quadrant of each distinct (frequency, depth) pair of the class is
// generated once per batched forward, into a table in the workspace that
// the column passes of every member scene read.
struct KernelClass {
    int M = 0, BS = 0, inv_r = 1;
    double dx = 0, dy = 0;
    const float2* tw = nullptr;          // twiddles of size M (a member plan's table)
    std::vector<double> f, z;            // distinct frequencies and depths
    double* d_f = nullptr;               // device copies (owned by the batch)
    double* d_z = nullptr;
    size_t off = 0;                      // workspace offset of the table [f][z][M/2+1][BS]
    bool on = false;                     // table within the limit and worth sharing
    size_t bytes() const { return f.size() * z.size() * (size_t)(M / 2 + 1) * BS * sizeof(float2); }
};

struct BatchScene {
    nursd_plan* p = nullptr;
    size_t off_P = 0, off_T1 = 0, off_U = 0, off_Bt = 0, off_Yt = 0, off_V = 0;
    int ZC = 1, rounds = 1;
    bool serial = false;     // propagated chunk by chunk with ordinary launches
    int kcls = -1;           // kernel class
    std::vector<int> kidx;   // [F][nz] plane of (b, iz) in the class table
    bool shared = false;     // reads the class table (set per configuration)
    size_t kidx_off = 0;     // byte offset of kidx in the table buffer
    bool multi = false;      // shared and chunk by chunk: column passes shared per kernel line
    bool zmono = false;      // plane depths map strictly monotonically onto the class depths
    size_t off_Ym = 0;       // [F][zr][M][ny] column-pass output of one depth round
};

struct BatchLaunch {
    int kind = 0, size = 0, fmax = 0;
    int var = 0;                                     // schedule variant of the grouped kernel
    int half = 0;                                    // row pass: every window within M/2
    int scene = -1;                                  // BK_SERIAL: scene propagated with ordinary launches
    size_t items = 0, prefix = 0, gridx = 0, item_of = 0;   // byte offsets in the table buffer
    int n = 0, total = 0, counter = -1;
    // BK_MULTI: last-pass chunks (scene, first plane, planes) of the round
    std::vector<std::array<int, 3>> p3;
};

// Relay lists of a scene binned for another spreading band height.
struct BatchLists {
    int nbands = 0;
    SpreadEntry* ent = nullptr;
    int* band_ptr = nullptr;
    int* wave_rng = nullptr;
};

struct nursd_batch {
    std::vector<BatchScene> sc;
    std::vector<KernelClass> kcls;
    // schedule variant of each grouped launch, keyed by (kind, size class)
    std::map<std::pair<int, int>, int> choice;
    std::vector<std::map<int, BatchLists>> lists;   // per scene: band rows -> lists
    std::vector<void*> owned;                       // device buffers of those lists
    std::vector<std::string> tuned;                 // what the kernel tuner picked, with times
    bool lists_missing = false;                     // a spreading tile without relay lists was asked for
    int multi_zr = 16;                              // class depths per round of the shared column passes
    int autotune = 0;
    BatchConfig cfg;                 // configuration in use
    std::vector<BatchConfig> cands;  // configurations the tuner times
    std::vector<int> tried;          // timed candidates (config_code) and their times
    std::vector<float> tried_ms;
    size_t ws_need = 0;              // caller workspace: covers every candidate
    size_t off_serial_Bt = 0, off_serial_Yt = 0;
    // pointers the captured graph was built for
    bool ready = false;
    const char* ws = nullptr;
    std::vector<const float*> hist;
    std::vector<float*> I;
    // small device tables owned by the batch, sized at creation for every candidate
    char* d_tab = nullptr;
    size_t tab_cap = 0;
    void* pinned = nullptr;          // staging buffer of the table upload
    hipEvent_t upload_done = nullptr;
    bool upload_pending = false;
    std::vector<char> tab;
    int* d_counters = nullptr;
    int counters_cap = 0;
    int n_counters = 0;              // work-queue counters in use (one per grouped launch)
    std::vector<BatchLaunch> launches;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~nursd_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        if (upload_done) (void)hipEventDestroy(upload_done);
        if (d_tab) (void)hipFree(d_tab);
        if (pinned) (void)hipHostFree(pinned);
        if (d_counters) (void)hipFree(d_counters);
        for (auto& k : kcls) {
            if (k.d_f) (void)hipFree(k.d_f);
            if (k.d_z) (void)hipFree(k.d_z);
        }
        for (void* d : owned) (void)hipFree(d);
    }
};

namespace {

template <typename T>
size_t tab_push(std::vector<char>& tab, const std::vector<T>& v) {
    size_t off = (tab.size() + 15) / 16 * 16;
    tab.resize(off + v.size() * sizeof(T));
    std::memcpy(tab.data() + off, v.data(), v.size() * sizeof(T));
    return off;
}

// Every scene is split into the same number of rounds so each round carries
// about 1/R of every scene's planes.
int batch_zc(const nursd_plan* p, int rounds) { return std::max(1, (p->nz + rounds - 1) / rounds); }

constexpr size_t kBatchScratchCap = 32ull << 30;      // propagation scratch limit of a tuner candidate
constexpr size_t kBatchKernelTableCap = 24ull << 30;  // kernel tables of all shared classes together
constexpr int kMaxGridY = 32768;                      // planes per kernel-table launch
constexpr size_t kBatchScratchDefault = 24ull << 30;  // default configuration without tuning

// Propagation scratch of the scenes propagated by grouped launches.
size_t batch_scratch_bytes(const nursd_batch* bt, int rounds, int serial_min_m) {
    size_t t = 0;
    for (const auto& sc : bt->sc) {
        const nursd_plan* p = sc.p;
        if (p->M >= serial_min_m) continue;
        const size_t zc = (size_t)batch_zc(p, rounds);
        t += (size_t)p->F * zc * ((size_t)(p->M / 2 + 1) * p->BS + (size_t)p->ny * p->M) * sizeof(float2);
    }
    return t;
}

// Workspace layout of configuration c (sets the scene offsets); returns its bytes.
size_t batch_layout(nursd_batch* bt, const BatchConfig& c) {
    size_t o = 0;
    const size_t c8 = sizeof(float2);
    size_t serial_bt = 0, serial_yt = 0;
    for (auto& k : bt->kcls)
        if (c.share && k.on) {
            k.off = o;
            o = align_up(o + k.bytes());
        }
    for (auto& sc : bt->sc) {
        nursd_plan* p = sc.p;
        sc.serial = p->M >= c.serial_min_m;
        sc.shared = c.share && bt->kcls[sc.kcls].on;
        sc.multi = sc.shared && sc.zmono;
        if (sc.serial && !sc.multi) {
            if (!sc.shared) serial_bt = std::max(serial_bt, (size_t)p->FC * p->ZC * (p->M / 2 + 1) * p->BS * c8);
            serial_yt = std::max(serial_yt, (size_t)p->FC * p->ZC * p->ny * p->M * c8);
        }
        if (sc.multi) {
            sc.off_Ym = o;
            o = align_up(o + (size_t)p->F * bt->multi_zr * p->M * p->ny * c8);
        }
        sc.ZC = batch_zc(p, c.rounds);
        sc.rounds = (sc.serial || sc.multi) ? 0 : (p->nz + sc.ZC - 1) / sc.ZC;
        sc.off_P = o;
        o = align_up(o + (size_t)p->F * p->L * c8);
        sc.off_T1 = o;
        o = align_up(o + (size_t)p->F * p->M * p->Mf * c8);
        sc.off_U = o;
        o = align_up(o + (size_t)p->F * p->M * p->M * c8);
        if (!sc.serial && !sc.multi) {
            sc.off_Bt = o;
            if (!sc.shared) o = align_up(o + (size_t)p->F * sc.ZC * (p->M / 2 + 1) * p->BS * c8);
            sc.off_Yt = o;
            o = align_up(o + (size_t)p->F * sc.ZC * p->ny * p->M * c8);
        }
        sc.off_V = o;
        o = align_up(o + (size_t)p->nvox() * c8);
    }
    bt->off_serial_Bt = o;
    o = align_up(o + serial_bt);
    bt->off_serial_Yt = o;
    o = align_up(o + serial_yt);
    return o;
}

// Schedule variants of the grouped launches: the plain launches' values by
// default (spreading tile of the plan, 4 lines per fine-y workgroup, 8 / 4 /
// 8 waves per block in the three propagation passes), else the tuner's pick.
int default_choice(int kind) {
    switch (kind) {
        case BK_FINEY: return 4;
        case BK_P1: return 8;
        case BK_P2: return 4;
        case BK_P3: return 8;
        default: return 0;
    }
}
int batch_choice(const nursd_batch* bt, int kind, int size) {
    auto it = bt->choice.find({kind, size});
    if (it != bt->choice.end()) return it->second;
    if (kind == BK_SPREAD) {             // the plans' own tile (the first plan of the size class)
        for (const auto& sc : bt->sc)
            if (sc.p->Mf == size) return sc.p->spread_var;
    }
    return default_choice(kind);
}
// Candidate variants of a (kind, size class) the tuner times.
std::vector<int> choice_candidates(const nursd_batch* bt, int kind, int size) {
    std::vector<int> v;
    switch (kind) {
        case BK_SPREAD:
            for (int c : {0, spread_var(1, 8), spread_var(1, 16), spread_var(2, 8), spread_var(4, 1), spread_var(4, 2),
                          spread_var(4, 4), spread_var(8, 1), spread_var(16, 1)}) {
                if (!spread_var_ok(size, c)) continue;
                const int br = spread_var_rows(c, size);
                bool have = true;
                for (size_t i = 0; i < bt->sc.size(); ++i) {
                    const nursd_plan* p = bt->sc[i].p;
                    if (p->Mf == size && br != spread_var_rows(p->spread_var, size) && !bt->lists[i].count(br))
                        have = false;
                }
                if (have && (c == 0 || c != spread_var(spread_band_rows(size), spread_freqs(size)))) v.push_back(c);
            }
            break;
        case BK_FINEY: v = {2, 4, 8}; break;
        case BK_P1: v = {4, 8}; break;
        case BK_P2: v = {2, 4, 8}; break;
        case BK_P3: v = {4, 8}; break;
        default: v = {0}; break;
    }
    return v;
}
// The finest variant of every grouped launch (the most virtual blocks), for
// sizing the table buffer.
void finest_choices(nursd_batch* bt) {
    bt->choice.clear();
    for (const auto& sc : bt->sc) {
        const int Mf = sc.p->Mf, M = sc.p->M;
        int sv = 0;
        for (int c : choice_candidates(bt, BK_SPREAD, Mf))
            if (c && (spread_var_rows(c, Mf) < spread_var_rows(sv, Mf) ||
                      (spread_var_rows(c, Mf) == spread_var_rows(sv, Mf) &&
                       spread_var_freqs(c, Mf) < spread_var_freqs(sv, Mf))))
                sv = c;
        bt->choice[{BK_SPREAD, Mf}] = sv;
        bt->choice[{BK_FINEY, Mf}] = 2;
        bt->choice[{BK_P1, M}] = 4;
        bt->choice[{BK_P2, M}] = 2;
        bt->choice[{BK_P3, M}] = 4;
    }
}

// Groups the scenes into kernel classes, lists each class's distinct
// frequencies and depths, maps every (b, iz) of a scene to its table plane
// and enables the table of a class when its scenes use each of its planes
// at least 1.5 times on average, largest savings first, within the limit.
int batch_kernel_classes(nursd_batch* bt) {
    for (auto& sc : bt->sc) {
        const nursd_plan* p = sc.p;
        int k = -1;
        for (size_t j = 0; j < bt->kcls.size() && k < 0; ++j) {
            const KernelClass& c = bt->kcls[j];
            if (c.M == p->M && c.BS == p->BS && c.inv_r == p->kernel_inv_r && c.dx == p->dx && c.dy == p->dy)
                k = (int)j;
        }
        if (k < 0) {
            KernelClass c;
            c.M = p->M;
            c.BS = p->BS;
            c.inv_r = p->kernel_inv_r;
            c.dx = p->dx;
            c.dy = p->dy;
            c.tw = p->tw(p->M);
            bt->kcls.push_back(c);
            k = (int)bt->kcls.size() - 1;
        }
        sc.kcls = k;
        KernelClass& c = bt->kcls[k];
        c.f.insert(c.f.end(), p->freqs.begin(), p->freqs.end());
        c.z.insert(c.z.end(), p->z.begin(), p->z.end());
    }
    std::vector<double> uses(bt->kcls.size(), 0.0);
    for (auto& c : bt->kcls) {
        std::sort(c.f.begin(), c.f.end());
        c.f.erase(std::unique(c.f.begin(), c.f.end()), c.f.end());
        std::sort(c.z.begin(), c.z.end());
        c.z.erase(std::unique(c.z.begin(), c.z.end()), c.z.end());
    }
    for (auto& sc : bt->sc) {
        const nursd_plan* p = sc.p;
        const KernelClass& c = bt->kcls[sc.kcls];
        sc.kidx.assign((size_t)p->F * p->nz, 0);
        for (int b = 0; b < p->F; ++b) {
            const int fi = (int)(std::lower_bound(c.f.begin(), c.f.end(), p->freqs[b]) - c.f.begin());
            for (int iz = 0; iz < p->nz; ++iz) {
                const int zi = (int)(std::lower_bound(c.z.begin(), c.z.end(), p->z[iz]) - c.z.begin());
                sc.kidx[(size_t)b * p->nz + iz] = fi * (int)c.z.size() + zi;
            }
        }
        uses[sc.kcls] += (double)p->F * p->nz;
        sc.zmono = true;
        for (int iz = 1; iz < p->nz; ++iz) {
            const int d = sc.kidx[iz] - sc.kidx[iz - 1];
            if (d == 0 || (iz > 1 && (d > 0) != (sc.kidx[1] > sc.kidx[0]))) sc.zmono = false;
        }
    }
    std::vector<int> order(bt->kcls.size());
    for (size_t j = 0; j < order.size(); ++j) order[j] = (int)j;
    auto saved = [&](int j) {
        const KernelClass& c = bt->kcls[j];
        return (uses[j] - (double)c.f.size() * c.z.size()) * (c.M / 2 + 1) * c.BS;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return saved(a) > saved(b); });
    size_t total = 0;
    for (int j : order) {
        KernelClass& c = bt->kcls[j];
        const double pairs = (double)c.f.size() * c.z.size();
        if (uses[j] < 1.5 * pairs || total + c.bytes() > kBatchKernelTableCap) continue;
        total += c.bytes();
        c.on = true;
        void* d = nullptr;
        HIP_TRY(hipMalloc(&d, c.f.size() * sizeof(double)));
        c.d_f = static_cast<double*>(d);
        HIP_TRY(hipMalloc(&d, c.z.size() * sizeof(double)));
        c.d_z = static_cast<double*>(d);
        HIP_TRY(hipMemcpy(c.d_f, c.f.data(), c.f.size() * sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c.d_z, c.z.data(), c.z.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    return NURSD_OK;
}

// Column-pass arguments of a chunk of a scene that reads its class table.
P2Args shared_cols_args(const nursd_batch* bt, const BatchScene& sc, const ChunkGeom& g, const float2* U,
                        float2* Yt, char* ws) {
    const KernelClass& k = bt->kcls[sc.kcls];
    P2Args a = cols_args(sc.p, g, reinterpret_cast<const float2*>(ws + k.off), U, Yt);
    a.kidx = reinterpret_cast<const int*>(reinterpret_cast<uintptr_t>(bt->d_tab) + sc.kidx_off);
    a.kz = sc.p->nz;
    return a;
}

// Kernel rows of class k for frequencies [f0, f1) at every class depth.
P1Args class_kernel_args(const nursd_batch* bt, int k, int f0, int f1, char* ws) {
    const KernelClass& kc = bt->kcls[k];
    ChunkGeom g{};
    g.b0 = f0;
    g.nb = f1 - f0;
    g.z0 = 0;
    g.nzc = (int)kc.z.size();
    g.f = kc.d_f;
    g.z = kc.d_z;
    g.dx = kc.dx;
    g.dy = kc.dy;
    g.uni = 0;
    const size_t plane = (size_t)(kc.M / 2 + 1) * kc.BS;
    P1Args a{g, reinterpret_cast<float2*>(ws + kc.off) + (size_t)f0 * kc.z.size() * plane, kc.M, kc.BS, kc.tw};
    a.plain = kc.inv_r ? 0 : 1;
    return a;
}

// Host side only: item tables and launch list of configuration c with the
// workspace at ws_base and the bound histogram / output pointers baked into
// the items.  Allocates nothing on the device.
void batch_tables(nursd_batch* bt, const BatchConfig& c, uintptr_t ws_base) {
    batch_layout(bt, c);
    char* ws = reinterpret_cast<char*>(ws_base);
    bt->tab.clear();
    bt->launches.clear();
    int max_rounds = 0;
    for (const auto& sc : bt->sc) max_rounds = std::max(max_rounds, sc.rounds);
    int counter = 0;
    // one grouped launch per (kind, size class); items are ordered by
    // descending work so the largest are dequeued first
    auto add = [&](int kind, int size, int fmax, int var, auto& items_in, std::vector<int>& gx_in,
                   std::vector<int>& gy_in, const std::vector<double>& work) {
        if (items_in.empty()) return;
        std::vector<size_t> ord(items_in.size());
        for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
        std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return work[a] > work[b]; });
        auto items = items_in;
        std::vector<int> gx(gx_in.size()), gy(gy_in.size());
        for (size_t i = 0; i < ord.size(); ++i) {
            items[i] = items_in[ord[i]];
            gx[i] = gx_in[ord[i]];
            gy[i] = gy_in[ord[i]];
        }
        BatchLaunch L;
        L.kind = kind;
        L.size = size;
        L.fmax = fmax;
        L.var = var;
        L.n = (int)items.size();
        std::vector<int> prefix(items.size() + 1, 0);
        for (size_t i = 0; i < items.size(); ++i) prefix[i + 1] = prefix[i] + gx[i] * gy[i];
        L.total = prefix.back();
        std::vector<int> item_of(L.total);
        for (size_t i = 0; i < items.size(); ++i)
            for (int v = prefix[i]; v < prefix[i + 1]; ++v) item_of[v] = (int)i;
        L.items = tab_push(bt->tab, items);
        L.prefix = tab_push(bt->tab, prefix);
        L.gridx = tab_push(bt->tab, gx);
        L.item_of = tab_push(bt->tab, item_of);
        L.counter = counter++;
        bt->launches.push_back(L);
    };
    std::vector<int> sizes;
    auto classes = [&](auto key) {
        std::vector<int> v;
        for (auto& sc : bt->sc) v.push_back(key(sc.p));
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        return v;
    };
    // step 1
    for (int T : classes([](nursd_plan* p) { return p->T; })) {
        std::vector<PhasorArgs> it;
        std::vector<int> gx, gy;
        std::vector<double> wk;
        int fmax = 0;
        for (size_t i = 0; i < bt->sc.size(); ++i) {
            nursd_plan* p = bt->sc[i].p;
            if (p->T != T) continue;
            PhasorArgs a{};
            a.hist = bt->hist.empty() ? nullptr : bt->hist[i];
            a.P = reinterpret_cast<float2*>(ws + bt->sc[i].off_P);
            a.L = p->L;
            a.T = p->T;
            a.F = p->F;
            a.bins = p->d_bins;
            a.wt = p->d_wt;
            a.tb = p->d_tb;
            a.tw = p->tw(p->T / 2);
            it.push_back(a);
            gx.push_back((p->L + phasor_group() - 1) / phasor_group());
            gy.push_back(1);
            wk.push_back((double)p->L);
            fmax = std::max(fmax, p->F);
        }
        add(BK_PHASOR, T, fmax, 0, it, gx, gy, wk);
    }
    // steps 2-3
    for (int Mf : classes([](nursd_plan* p) { return p->Mf; })) {
        std::vector<SpreadArgs> it;
        std::vector<FineYArgs> it2;
        std::vector<int> gx, gy, gx2, gy2;
        std::vector<double> wk;
        const int sv = batch_choice(bt, BK_SPREAD, Mf), nl = batch_choice(bt, BK_FINEY, Mf);
        const int BR = spread_var_rows(sv, Mf), NF = spread_var_freqs(sv, Mf);
        for (size_t i = 0; i < bt->sc.size(); ++i) {
            BatchScene& sc = bt->sc[i];
            nursd_plan* p = sc.p;
            if (p->Mf != Mf) continue;
            SpreadArgs a{};
            a.P = reinterpret_cast<float2*>(ws + sc.off_P);
            a.wts = p->d_w;
            a.ent = p->d_ent;
            a.band_ptr = p->d_band_ptr;
            a.wave_rng = p->d_wave_rng;
            int nbands = p->nbands;
            if (BR != spread_var_rows(p->spread_var, Mf)) {     // lists the batch binned for this band height
                auto li = bt->lists[i].find(BR);
                if (li == bt->lists[i].end()) {
                    bt->lists_missing = true;        // reported by batch_upload / creation
                } else {
                    a.ent = li->second.ent;
                    a.band_ptr = li->second.band_ptr;
                    a.wave_rng = li->second.wave_rng;
                    nbands = li->second.nbands;
                }
            }
            a.T1 = reinterpret_cast<float2*>(ws + sc.off_T1);
            a.decx = p->d_decx;
            a.tw = p->tw(Mf);
            a.M = p->M;
            a.Mf = Mf;
            a.L = p->L;
            a.w = p->w;
            a.beta = (float)p->beta;
            a.half_w = 0.5f * p->w;
            a.b0 = 0;
            a.nb = p->F;
            it.push_back(a);
            gx.push_back(nbands);
            gy.push_back((p->F + NF - 1) / NF);
            FineYArgs f{};
            f.T1 = a.T1;
            f.U = reinterpret_cast<float2*>(ws + sc.off_U);
            f.decy = p->d_decy;
            f.tw = p->tw(Mf);
            f.M = p->M;
            f.Mf = Mf;
            f.b0 = 0;
            f.nb = p->F;
            f.br = BR;
            it2.push_back(f);
            gx2.push_back(p->M / nl);
            gy2.push_back(p->F);
            wk.push_back((double)p->F * p->L);
        }
        add(BK_SPREAD, Mf, 0, sv, it, gx, gy, wk);
        add(BK_FINEY, Mf, 0, nl, it2, gx2, gy2, wk);
    }
    // kernel tables: the quadrant of every distinct (frequency, depth) pair
    // of each shared kernel class, before any column pass reads them
    for (size_t k = 0; k < bt->kcls.size(); ++k) {
        if (!(c.share && bt->kcls[k].on)) continue;
        BatchLaunch L;
        L.kind = BK_KTAB;
        L.scene = (int)k;
        bt->launches.push_back(L);
    }
    for (auto& sc : bt->sc)
        if (sc.shared) sc.kidx_off = tab_push(bt->tab, sc.kidx);
    // steps 4-7, round by round
    const std::vector<int> Ms = classes([](nursd_plan* p) { return p->M; });
    for (int r = 0; r < max_rounds; ++r) {
        for (int M : Ms) {
            std::vector<P1Args> i1;
            std::vector<P2Args> i2;
            std::vector<P3Args> i3;
            std::vector<int> g1x, g1y, g2x, g2y, g3x, g3y;
            std::vector<double> w1, w12, w3;
            const int nw1 = batch_choice(bt, BK_P1, M), nw2 = batch_choice(bt, BK_P2, M);
            const int nw3 = batch_choice(bt, BK_P3, M);
            bool half = true;       // one row-pass variant per launch: every window within M/2
            bool halfy = true;      // the same for the column pass, along y
            for (const BatchScene& sc : bt->sc)
                if (sc.p->M == M && r < sc.rounds) {
                    half = half && 2 * sc.p->nx * sc.p->q <= M;
                    halfy = halfy && 2 * sc.p->ny * sc.p->q <= M;
                }
            for (size_t i = 0; i < bt->sc.size(); ++i) {
                BatchScene& sc = bt->sc[i];
                nursd_plan* p = sc.p;
                if (p->M != M || r >= sc.rounds) continue;
                const int z0 = r * sc.ZC, nzc = std::min(sc.ZC, p->nz - z0);
                const ChunkGeom g = chunk_geom(p, 0, p->F, z0, nzc);
                float2* Bt = reinterpret_cast<float2*>(ws + sc.off_Bt);
                float2* Yt = reinterpret_cast<float2*>(ws + sc.off_Yt);
                const float2* U = reinterpret_cast<const float2*>(ws + sc.off_U);
                if (sc.shared) {
                    i2.push_back(shared_cols_args(bt, sc, g, U, Yt, ws));
                } else {
                    i1.push_back(kernel_args(p, g, Bt));
                    g1x.push_back(grid_x_kernel_rows(M, nw1));
                    g1y.push_back(p->F * nzc);
                    w1.push_back((double)p->F * nzc);
                    i2.push_back(cols_args(p, g, Bt, U, Yt));
                }
                g2x.push_back(grid_x_propagate_cols(M, nw2));
                g2y.push_back(p->F * nzc);
                P3Args a3 = rows_args(p, g, Yt, reinterpret_cast<float2*>(ws + sc.off_V), bt->I.empty() ? nullptr : bt->I[i], 0, p->F);
                i3.push_back(a3);
                const int rb = rows_per_block_propagate(M, nw3);
                g3x.push_back((p->ny + rb - 1) / rb);
                g3y.push_back(nzc);
                w12.push_back((double)p->F * nzc);
                w3.push_back((double)p->F);      // per block: one pass per frequency
            }
            add(BK_P1, M, 0, nw1, i1, g1x, g1y, w1);
            add(BK_P2, M, 0, nw2, i2, g2x, g2y, w12);
            if (!i2.empty()) bt->launches.back().half = halfy ? 1 : 0;
            add(BK_P3, M, 0, nw3, i3, g3x, g3y, w3);
            if (!i3.empty()) bt->launches.back().half = half ? 1 : 0;
        }
    }
    // chunk-by-chunk scenes of shared classes: rounds of class depths, each
    // one column pass per kernel line for all the class's scenes, then the
    // scenes' last passes with ordinary launches
    for (size_t k = 0; k < bt->kcls.size(); ++k) {
        const KernelClass& kc = bt->kcls[k];
        std::vector<int> mem;
        for (size_t i = 0; i < bt->sc.size(); ++i)
            if (bt->sc[i].multi && bt->sc[i].kcls == (int)k) mem.push_back((int)i);
        if (mem.empty()) continue;
        const int nzk = (int)kc.z.size(), zr = bt->multi_zr;
        for (int zi0 = 0; zi0 < nzk; zi0 += zr) {
            const int zi1 = std::min(nzk, zi0 + zr);
            std::map<int, std::vector<P2MUser>> users;     // table plane -> users
            BatchLaunch L;
            L.kind = BK_MULTI;
            L.scene = (int)k;
            L.half = 1;             // every user's window within M/2 rows
            for (int i : mem) {
                const BatchScene& sc = bt->sc[i];
                const nursd_plan* p = sc.p;
                int iz0 = -1, iz1 = -1;
                for (int iz = 0; iz < p->nz; ++iz) {
                    const int zi = sc.kidx[iz] % nzk;             // b = 0 row of the plane map
                    if (zi >= zi0 && zi < zi1) {
                        if (iz0 < 0) iz0 = iz;
                        iz1 = iz + 1;
                    }
                }
                if (iz0 < 0) continue;
                const int nzr = iz1 - iz0;
                for (int b = 0; b < p->F; ++b)
                    for (int iz = iz0; iz < iz1; ++iz) {
                        P2MUser u;
                        u.U = reinterpret_cast<const float2*>(ws + sc.off_U) + (size_t)b * p->M * p->M;
                        u.Yt = reinterpret_cast<float2*>(ws + sc.off_Ym) + ((size_t)b * nzr + (iz - iz0)) * p->M * p->ny;
                        u.ny = p->ny;
                        u.q = p->q;
                        users[sc.kidx[(size_t)b * p->nz + iz]].push_back(u);
                        if (2 * p->ny * p->q > p->M) L.half = 0;
                    }
                L.p3.push_back({i, iz0, nzr});
            }
            // last passes of the round: chunk-by-chunk scenes as ordinary
            // launches (listed in L.p3), the others in one grouped launch
            std::vector<P3Args> g3;
            std::vector<int> g3x, g3y;
            std::vector<double> w3;
            bool half = true;
            std::vector<std::array<int, 3>> ord;
            for (const auto& t : L.p3) {
                const BatchScene& sc = bt->sc[t[0]];
                const nursd_plan* p = sc.p;
                if (sc.serial) {
                    ord.push_back(t);
                    continue;
                }
                half = half && 2 * p->nx * p->q <= p->M;
            }
            const int nw3 = batch_choice(bt, BK_P3, kc.M);
            for (const auto& t : L.p3) {
                const BatchScene& sc = bt->sc[t[0]];
                nursd_plan* p = sc.p;
                if (sc.serial) continue;
                // one item per scene and round over all its frequencies: the
                // items of a grouped launch run concurrently, so frequency
                // chunks of the same planes must not be separate items
                float2* Ym = reinterpret_cast<float2*>(ws + sc.off_Ym);
                const ChunkGeom g = chunk_geom(p, 0, p->F, t[1], t[2]);
                g3.push_back(rows_args(p, g, Ym, reinterpret_cast<float2*>(ws + sc.off_V),
                                       bt->I.empty() ? nullptr : bt->I[t[0]], 0, p->F));
                const int rb = rows_per_block_propagate(p->M, nw3);
                g3x.push_back((p->ny + rb - 1) / rb);
                g3y.push_back(t[2]);
                w3.push_back((double)p->F);
            }
            L.p3 = ord;
            std::vector<int> kp, ptr(1, 0);
            std::vector<P2MUser> flat;
            for (auto& kv : users) {
                kp.push_back(kv.first);
                flat.insert(flat.end(), kv.second.begin(), kv.second.end());
                ptr.push_back((int)flat.size());
            }
            // work blocks: for each frequency's run of items (table planes
            // are frequency-major), eight kx blocks at a time, interleaved
            // so that one kx block's depths fall on one XCD
            const int kxb = grid_x_propagate_cols_multi(kc.M);
            std::vector<int2> blk;
            for (size_t i0 = 0; i0 < kp.size();) {
                size_t i1 = i0;
                while (i1 < kp.size() && kp[i1] / nzk == kp[i0] / nzk) ++i1;
                for (int c0 = 0; c0 < kxb; c0 += kXcds)
                    for (size_t i = i0; i < i1; ++i)
                        for (int x = c0; x < std::min(kxb, c0 + kXcds); ++x) blk.push_back(make_int2((int)i, x));
                i0 = i1;
            }
            L.n = (int)kp.size();
            L.total = (int)blk.size();
            L.items = tab_push(bt->tab, kp);
            L.prefix = tab_push(bt->tab, ptr);
            L.gridx = tab_push(bt->tab, flat);
            L.item_of = tab_push(bt->tab, blk);
            bt->launches.push_back(L);
            if (!g3.empty()) {
                add(BK_P3, kc.M, 0, nw3, g3, g3x, g3y, w3);
                bt->launches.back().half = half ? 1 : 0;
            }
        }
    }
    // large-transform scenes: ordinary chunked launches, largest first
    {
        std::vector<int> order;
        for (size_t i = 0; i < bt->sc.size(); ++i)
            if (bt->sc[i].serial && !bt->sc[i].multi) order.push_back((int)i);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            const nursd_plan *pa = bt->sc[a].p, *pb = bt->sc[b].p;
            return (double)pa->F * pa->nz * pa->M * pa->M > (double)pb->F * pb->nz * pb->M * pb->M;
        });
        for (int i : order) {
            BatchLaunch L;
            L.kind = BK_SERIAL;
            L.scene = i;
            bt->launches.push_back(L);
        }
    }
    bt->n_counters = counter;
}

// Table bytes and counters configuration c needs.
void batch_table_size(nursd_batch* bt, const BatchConfig& c, size_t* tab_bytes, int* counters) {
    batch_tables(bt, c, kAlign);
    *tab_bytes = bt->tab.size();
    *counters = bt->n_counters;
}

template <typename A>
Group<A> group_of(nursd_batch* bt, const BatchLaunch& L) {
    Group<A> g;
    g.items = reinterpret_cast<const A*>(bt->d_tab + L.items);
    g.prefix = reinterpret_cast<const int*>(bt->d_tab + L.prefix);
    g.gridx = reinterpret_cast<const int*>(bt->d_tab + L.gridx);
    g.item_of = reinterpret_cast<const int*>(bt->d_tab + L.item_of);
    g.n = L.n;
    g.total = L.total;
    g.counter = bt->d_counters + L.counter;
    g.mode = bt->cfg.sched;
    return g;
}

// Timing hook of the kernel tuner: events around every grouped launch of
// one (kind, size class) in an eager run of the launch sequence.
struct LaunchTimer {
    int kind = -1, size = 0;
    std::vector<hipEvent_t> ev;    // pairs, created on demand
    size_t used = 0;
    ~LaunchTimer() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    hipError_t mark(hipStream_t s) {
        if (used == ev.size()) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            ev.push_back(e);
        }
        return hipEventRecord(ev[used++], s);
    }
    hipError_t total_ms(float* ms) {
        *ms = 0.f;
        for (size_t i = 0; i + 1 < used; i += 2) {
            float t = 0.f;
            hipError_t r = hipEventSynchronize(ev[i + 1]);
            if (r == hipSuccess) r = hipEventElapsedTime(&t, ev[i], ev[i + 1]);
            if (r != hipSuccess) return r;
            *ms += t;
        }
        return hipSuccess;
    }
};

int batch_enqueue(nursd_batch* bt, hipStream_t s, LaunchTimer* tm = nullptr) {
    // One work-queue counter per grouped launch; scenes propagated with
    // ordinary launches have none.
    for (const BatchLaunch& L : bt->launches)
        if (L.kind != BK_SERIAL && L.kind != BK_KTAB && L.kind != BK_MULTI &&
            (L.counter < 0 || L.counter >= bt->n_counters || bt->n_counters > bt->counters_cap))
            return fail(NURSD_ERR_ARG, "batch launch table refers to a counter outside the counter buffer");
    if (bt->n_counters > 0) HIP_TRY(launch_zero_counters(bt->d_counters, bt->n_counters, s));
    char* ws = const_cast<char*>(bt->ws);
    for (const BatchLaunch& L : bt->launches) {
        if (L.kind == BK_MULTI) {
            const KernelClass& kc = bt->kcls[L.scene];
            P2MArgs ma{};
            ma.Bt = reinterpret_cast<const float2*>(ws + kc.off);
            ma.kp = reinterpret_cast<const int*>(bt->d_tab + L.items);
            ma.user_ptr = reinterpret_cast<const int*>(bt->d_tab + L.prefix);
            ma.users = reinterpret_cast<const P2MUser*>(bt->d_tab + L.gridx);
            ma.blk = reinterpret_cast<const int2*>(bt->d_tab + L.item_of);
            ma.M = kc.M;
            ma.BS = kc.BS;
            ma.tw = kc.tw;
            HIP_TRY(launch_propagate_cols_multi(ma, L.total, L.half != 0, s));
            for (const auto& t : L.p3) {
                const BatchScene& sc = bt->sc[t[0]];
                nursd_plan* p = sc.p;
                float2* Ym = reinterpret_cast<float2*>(ws + sc.off_Ym);
                float2* V = reinterpret_cast<float2*>(ws + sc.off_V);
                for (int b0 = 0; b0 < p->F; b0 += p->FC) {
                    const int nb = std::min(p->FC, p->F - b0);
                    const ChunkGeom g = chunk_geom(p, b0, nb, t[1], t[2]);
                    HIP_TRY(launch_propagate_rows(
                        rows_args(p, g, Ym + (size_t)b0 * t[2] * p->M * p->ny, V, bt->I[t[0]], b0, nb), s));
                }
            }
            continue;
        }
        if (L.kind == BK_KTAB) {
            const int nf = (int)bt->kcls[L.scene].f.size(), nzk = (int)bt->kcls[L.scene].z.size();
            const int fstep = std::max(1, kMaxGridY / std::max(1, nzk));
            for (int f0 = 0; f0 < nf; f0 += fstep)
                HIP_TRY(launch_kernel_rows(class_kernel_args(bt, L.scene, f0, std::min(nf, f0 + fstep), ws), s));
            continue;
        }
        if (L.kind == BK_SERIAL) {
            const BatchScene& sc = bt->sc[L.scene];
            nursd_plan* p = sc.p;
            float2* Bt = reinterpret_cast<float2*>(ws + bt->off_serial_Bt);
            float2* Yt = reinterpret_cast<float2*>(ws + bt->off_serial_Yt);
            const float2* U = reinterpret_cast<const float2*>(ws + sc.off_U);
            float2* V = reinterpret_cast<float2*>(ws + sc.off_V);
            for (int b0 = 0; b0 < p->F; b0 += p->FC) {
                const int nb = std::min(p->FC, p->F - b0);
                for (int z0 = 0; z0 < p->nz; z0 += p->ZC) {
                    const int nzc = std::min(p->ZC, p->nz - z0);
                    const ChunkGeom g = chunk_geom(p, b0, nb, z0, nzc);
                    if (sc.shared) {
                        HIP_TRY(launch_propagate_cols(shared_cols_args(bt, sc, g, U, Yt, ws), s));
                    } else {
                        HIP_TRY(launch_kernel_rows(kernel_args(p, g, Bt), s));
                        HIP_TRY(launch_propagate_cols(cols_args(p, g, Bt, U, Yt), s));
                    }
                    HIP_TRY(launch_propagate_rows(rows_args(p, g, Yt, V, bt->I[L.scene], b0, nb), s));
                }
            }
            continue;
        }
        const bool timed_launch = tm && L.kind == tm->kind && L.size == tm->size;
        if (timed_launch) HIP_TRY(tm->mark(s));
        switch (L.kind) {
            case BK_PHASOR: HIP_TRY(launch_phasor_grouped(L.size, L.fmax, group_of<PhasorArgs>(bt, L), s)); break;
            case BK_SPREAD: HIP_TRY(launch_spread_xfft_grouped(L.size, L.var, group_of<SpreadArgs>(bt, L), s)); break;
            case BK_FINEY: HIP_TRY(launch_fine_y_grouped(L.size, L.var, group_of<FineYArgs>(bt, L), s)); break;
            case BK_P1: HIP_TRY(launch_kernel_rows_grouped(L.size, L.var, group_of<P1Args>(bt, L), s)); break;
            case BK_P2:
                HIP_TRY(launch_propagate_cols_grouped(L.size, L.half != 0, L.var, group_of<P2Args>(bt, L), s));
                break;
            default:
                HIP_TRY(launch_propagate_rows_grouped(L.size, L.half != 0, L.var, group_of<P3Args>(bt, L), s));
                break;
        }
        if (timed_launch) HIP_TRY(tm->mark(s));
    }
    return NURSD_OK;
}

int batch_capture(nursd_batch* bt) {
    if (bt->exec) HIP_TRY(hipGraphExecDestroy(bt->exec));
    if (bt->graph) HIP_TRY(hipGraphDestroy(bt->graph));
    bt->exec = nullptr;
    bt->graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(bt->cap, hipStreamCaptureModeThreadLocal));
    int rc = batch_enqueue(bt, bt->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(bt->cap, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(NURSD_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    bt->graph = g;
    HIP_TRY(hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0));
    return NURSD_OK;
}

// Tables of the current configuration for the given workspace and the bound
// histogram / output pointers: built on the host, copied to the batch's
// device table buffer on `s` through the pinned staging buffer (the host
// waits only for this batch's previous table copy to leave the staging
// buffer), then the launch sequence is captured as a graph.
int batch_upload(nursd_batch* bt, const char* ws, hipStream_t s) {
    bt->lists_missing = false;
    batch_tables(bt, bt->cfg, reinterpret_cast<uintptr_t>(ws));
    if (bt->lists_missing) return fail(NURSD_ERR_ARG, "batch spreading tile without binned relay lists");
    if (bt->tab.size() > bt->tab_cap || bt->n_counters > bt->counters_cap)
        return fail(NURSD_ERR_ARG, "batch tables exceed the buffers sized at creation");
    if (bt->upload_pending) HIP_TRY(hipEventSynchronize(bt->upload_done));
    if (!bt->tab.empty()) {
        std::memcpy(bt->pinned, bt->tab.data(), bt->tab.size());
        HIP_TRY(hipMemcpyAsync(bt->d_tab, bt->pinned, bt->tab.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipEventRecord(bt->upload_done, s));
        bt->upload_pending = true;
    }
    bt->ws = ws;
    return NURSD_OK;
}

int batch_bind(nursd_batch* bt, const char* ws, hipStream_t s) {
    bt->ready = false;
    int rc = batch_upload(bt, ws, s);
    if (rc) return rc;
    rc = batch_capture(bt);
    if (rc) return rc;
    bt->ready = true;
    return NURSD_OK;
}

int batch_check_io(nursd_batch* bt, const float* const* hist, float* const* I, void* ws, size_t ws_bytes,
                   bool* changed) {
    if (!hist || !I) return fail(NURSD_ERR_ARG, "NULL argument");
    if (!ws) return fail(NURSD_ERR_WORKSPACE, "workspace pointer is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(NURSD_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < bt->ws_need)
        return fail(NURSD_ERR_WORKSPACE, "batch workspace too small: need " + std::to_string(bt->ws_need) + " bytes");
    const int n = (int)bt->sc.size();
    for (int i = 0; i < n; ++i) {
        if (!hist[i] || !I[i]) return fail(NURSD_ERR_ARG, "NULL histogram or output pointer");
        if (reinterpret_cast<uintptr_t>(hist[i]) & 7) return fail(NURSD_ERR_ARG, "histograms must be 8-byte aligned");
    }
    bool ch = !bt->ready || bt->ws != ws;
    for (int i = 0; i < n; ++i) {
        if (hist[i] != bt->hist[i] || I[i] != bt->I[i]) ch = true;
        bt->hist[i] = hist[i];
        bt->I[i] = I[i];
    }
    *changed = ch;
    return NURSD_OK;
}

}  // namespace

namespace {

// Process-wide picks of the kernel tuner, keyed by (kind, size class, work
// bucket = floor(log2) of the launch's total work items), so a later batch
// of the same shape reuses them without timing.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tune_cache;

const char* kind_name(int kind) {
    switch (kind) {
        case BK_SPREAD: return "spread";
        case BK_FINEY: return "fine_y";
        case BK_P1: return "kernel_rows";
        case BK_P2: return "propagate_cols";
        case BK_P3: return "propagate_rows";
        default: return "other";
    }
}

std::string choice_name(int kind, int size, int var) {
    if (kind == BK_SPREAD)
        return "band_rows=" + std::to_string(spread_var_rows(var, size)) +
               ",freqs_per_block=" + std::to_string(spread_var_freqs(var, size));
    if (kind == BK_FINEY) return "lines_per_block=" + std::to_string(var);
    return "waves_per_block=" + std::to_string(var);
}

// Second tuner stage: for the chosen configuration, each grouped launch
// class (kind, size) in turn tries its schedule variants (spreading tile;
// lines or waves per block of the transforms), timed with events around
// that class's launches in an eager run of the whole sequence (best of
// two runs), and keeps the fastest.  Picks are cached per process.
int batch_tune_kernels(nursd_batch* bt, const char* ws, hipStream_t s) {
    bt->tuned.clear();
    int rc = batch_upload(bt, ws, s);
    if (rc) return rc;
    // the grouped launch classes of the chosen configuration, with the
    // log2 of their virtual blocks as the work bucket
    std::vector<std::tuple<int, int, int>> keys;      // kind, size, work bucket
    {
        std::map<std::pair<int, int>, double> work;
        for (const BatchLaunch& L : bt->launches)
            if (L.kind == BK_SPREAD || L.kind == BK_FINEY || L.kind == BK_P1 || L.kind == BK_P2 || L.kind == BK_P3)
                work[{L.kind, L.size}] += (double)L.total;
        for (const auto& kv : work)
            keys.emplace_back(kv.first.first, kv.first.second, (int)std::floor(std::log2(std::max(1.0, kv.second))));
    }
    for (const auto& key : keys) {
        const int kind = std::get<0>(key), size = std::get<1>(key);
        const std::vector<int> cand = choice_candidates(bt, kind, size);
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end() && std::find(cand.begin(), cand.end(), it->second) != cand.end()) {
                bt->choice[{kind, size}] = it->second;
                bt->tuned.push_back(std::string(kind_name(kind)) + "/" + std::to_string(size) + ": " +
                                    choice_name(kind, size, it->second) + " (cached)");
                continue;
            }
        }
        int best_v = batch_choice(bt, kind, size);
        float best = 1e30f, def_ms = -1.f;
        for (int v : cand) {
            bt->choice[{kind, size}] = v;
            if ((rc = batch_upload(bt, ws, s))) return rc;
            float ms = 1e30f;
            for (int rep = 0; rep < 2; ++rep) {
                LaunchTimer tm;
                tm.kind = kind;
                tm.size = size;
                if ((rc = batch_enqueue(bt, s, &tm))) return rc;
                float t = 0.f;
                const hipError_t e = tm.total_ms(&t);
                if (e != hipSuccess) return fail(NURSD_ERR_HIP, std::string("kernel tuner: ") + hipGetErrorString(e));
                ms = std::min(ms, t);
            }
            if (v == default_choice(kind)) def_ms = ms;
            if (ms < best) {
                best = ms;
                best_v = v;
            }
        }
        bt->choice[{kind, size}] = best_v;
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            g_tune_cache[key] = best_v;
        }
        char buf[96];
        std::snprintf(buf, sizeof buf, " (%.3f ms, default %.3f ms)", best, def_ms);
        bt->tuned.push_back(std::string(kind_name(kind)) + "/" + std::to_string(size) + ": " +
                            choice_name(kind, size, best_v) + buf);
    }
    return NURSD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free forward.  The array's name is a
// host-side stand-in in host code: its device address comes from
// hipGetSymbolAddress, once per device with that device current, and only
// that address is ever passed to kernels.
constexpr size_t kStaticScratchBytes = NURSD_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

int static_scratch(void** out) {
    *out = nullptr;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(NURSD_ERR_HIP, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(NURSD_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return NURSD_OK;
}
}  // namespace

extern "C" {

void nursd_default_options(nursd_wavelet* wl, nursd_geometry* geo, nursd_options* opt) {
    if (wl) {
        std::memset(wl, 0, sizeof(*wl));
        wl->sigma_rel = 0.2;
        wl->coherent = 1;
        wl->kernel_inv_r = 1;
    }
    if (geo) std::memset(geo, 0, sizeof(*geo));
    if (opt) {
        std::memset(opt, 0, sizeof(*opt));
        opt->pad = 2.0;
        opt->sigma_os = 2.0;
        opt->tol = 1e-6;
        opt->upsample_q = 1;
    }
}

static int nursd_plan_create_body(const nursd_wavelet* wl, const nursd_geometry* geo, const nursd_options* opt,
                      const float* relay_xy_dev, void* stream, nursd_plan** out) {
    if (!out) return fail(NURSD_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!wl || !geo || !opt || !relay_xy_dev) return fail(NURSD_ERR_ARG, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto p = new nursd_plan();
    auto bail = [&](int rc) {
        delete p;
        return rc;
    };
    // wavelet and frequency bins
    if (!(wl->lambda_c > 0) || !(wl->dt > 0) || wl->n_time < 2 || wl->n_freq < 1)
        return bail(fail(NURSD_ERR_ARG, "invalid wavelet parameters"));
    p->F = wl->n_freq;
    p->T = wl->n_time;
    p->lambda_c = wl->lambda_c;
    p->sigma_rel = wl->sigma_rel;
    p->dt = wl->dt;
    p->t0 = wl->t0;
    p->coherent = wl->coherent ? 1 : 0;
    p->kernel_inv_r = wl->kernel_inv_r ? 1 : 0;
    const double df = 1.0 / (p->T * p->dt);
    const double fc = kC / p->lambda_c;
    if (wl->bins) {
        p->bins.assign(wl->bins, wl->bins + p->F);
    } else {
        const long k0 = std::lround(fc / df);
        for (int j = 0; j < p->F; ++j) p->bins.push_back((int)(k0 - p->F / 2 + j));
    }
    for (int b : p->bins)
        if (b <= 0 || 2L * b >= p->T) return bail(fail(NURSD_ERR_ARG, "frequency bin outside (0, T/2)"));
    for (int b : p->bins) p->freqs.push_back(b * df);
    // geometry
    p->mode = geo->mode;
    if (p->mode != NURSD_MODE_GRID && p->mode != NURSD_MODE_POINTS && p->mode != NURSD_MODE_SRSD &&
        p->mode != NURSD_MODE_SRSD_POINTS && p->mode != NURSD_MODE_GRID3D)
        return bail(fail(NURSD_ERR_ARG, "unknown mode"));
    if (geo->nz < 1 || !geo->z) return bail(fail(NURSD_ERR_ARG, "no planes"));
    p->nz = geo->nz;
    p->z.assign(geo->z, geo->z + geo->nz);
    for (double zz : p->z)
        if (!(zz > 0)) return bail(fail(NURSD_ERR_GEOMETRY, "plane depth must be > 0"));
    p->x0 = geo->x0;
    p->y0 = geo->y0;
    p->vdx = geo->dx;
    p->vdy = geo->dy;
    p->nx = geo->nx;
    p->ny = geo->ny;
    std::memcpy(p->xp, geo->xp, sizeof(p->xp));
    if (!(geo->dx > 0) || !(geo->dy > 0)) return bail(fail(NURSD_ERR_ARG, "pitch must be > 0"));
    if (opt->n_relay < 1) return bail(fail(NURSD_ERR_ARG, "n_relay must be >= 1"));
    p->L = opt->n_relay;
    p->pad = opt->pad > 0 ? opt->pad : 2.0;
    if (p->pad < 1.0) return bail(fail(NURSD_ERR_ARG, "pad must be >= 1"));
    if (opt->sigma_os != 0.0 && opt->sigma_os != 2.0)
        return bail(fail(NURSD_ERR_UNSUPPORTED_SIZE, "only NUFFT oversampling 2 is supported"));
    const double tol = opt->tol > 0 ? opt->tol : 1e-6;
    p->w = std::min(8, std::max(2, (int)std::ceil(std::log10(1.0 / tol)) + 1));
    p->beta = 2.30 * p->w;
    p->q = opt->upsample_q > 0 ? opt->upsample_q : 1;
    if (p->q > 16) return bail(fail(NURSD_ERR_ARG, "upsample_q must be in [1, 16]"));
    if (p->q > 1 && (p->mode == NURSD_MODE_SRSD || p->mode == NURSD_MODE_SRSD_POINTS))
        return bail(fail(NURSD_ERR_UNSUPPORTED_SIZE, "the scaled RSD needs upsample_q = 1"));

    std::vector<float> rxy;
    int rc = read_points(relay_xy_dev, (size_t)p->L * 2, rxy, s);
    if (rc) return bail(rc);
    for (float v : rxy)
        if (!std::isfinite(v)) return bail(fail(NURSD_ERR_GEOMETRY, "non-finite relay position"));

    double vlo[2], vhi[2], mmin = 0;
    std::vector<float> vxy;
    if (p->mode == NURSD_MODE_GRID || p->mode == NURSD_MODE_GRID3D || p->scaled()) {
        if (p->nx < 1 || p->ny < 1) return bail(fail(NURSD_ERR_ARG, "nx, ny must be >= 1"));
        // grid pitch vdx / q; voxel ix is grid point ix q - (nx q)/2 around c
        p->dx = p->vdx / p->q;
        p->dy = p->vdy / p->q;
        p->cx = p->x0 + ((p->nx * p->q) / 2) * p->dx;
        p->cy = p->y0 + ((p->ny * p->q) / 2) * p->dy;
        vlo[0] = p->x0;
        vlo[1] = p->y0;
        vhi[0] = p->x0 + (p->nx - 1) * p->vdx;
        vhi[1] = p->y0 + (p->ny - 1) * p->vdy;
        mmin = p->pad * std::max(p->nx, p->ny) * p->q;
        if (p->scaled()) {
            p->zref = geo->zref;
            for (int i = 0; i < p->nz; ++i) {
                const double a = geo->alpha ? geo->alpha[i] : geo->zref / p->z[i];
                if (!(a > 0 && a <= 1)) return bail(fail(NURSD_ERR_GEOMETRY, "SRSD scale alpha must be in (0, 1]"));
                p->alpha.push_back(a);
            }
        }
        if (p->mode == NURSD_MODE_SRSD_POINTS) {
            if (!geo->plane_ptr || !geo->voxel_xy_dev)
                return bail(fail(NURSD_ERR_ARG, "SRSD_POINTS mode needs plane_ptr and voxel_xy_dev"));
            if ((rc = read_voxel_lists(p, geo, vxy, s))) return bail(rc);
        }
    } else {
        if (!geo->plane_ptr || !geo->voxel_xy_dev) return bail(fail(NURSD_ERR_ARG, "POINTS mode needs plane_ptr and voxel_xy_dev"));
        p->dx = p->vdx / p->q;
        p->dy = p->vdy / p->q;
        if ((rc = read_voxel_lists(p, geo, vxy, s))) return bail(rc);
        const int V = p->plane_ptr.back();
        double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
        for (int i = 0; i < V; ++i)
            for (int a = 0; a < 2; ++a) {
                vlo[a] = std::min(i ? vlo[a] : 1e300, (double)vxy[2 * i + a]);
                vhi[a] = std::max(i ? vhi[a] : -1e300, (double)vxy[2 * i + a]);
            }
        for (int a = 0; a < 2; ++a) {
            lo[a] = vlo[a];
            hi[a] = vhi[a];
        }
        for (int l = 0; l < p->L; ++l)
            for (int a = 0; a < 2; ++a) {
                lo[a] = std::min(lo[a], (double)rxy[2 * l + a]);
                hi[a] = std::max(hi[a], (double)rxy[2 * l + a]);
            }
        p->cx = 0.5 * (lo[0] + hi[0]);
        p->cy = 0.5 * (lo[1] + hi[1]);
    }
    p->M = 0;
    if (opt->M > 0 && std::find(std::begin(kSupportedM), std::end(kSupportedM), opt->M) == std::end(kSupportedM))
        return bail(fail(NURSD_ERR_UNSUPPORTED_SIZE, "M must be a power of two in [64, 1024]"));
    for (int Mc : kSupportedM) {
        if (opt->M > 0 && Mc != opt->M) continue;
        if (Mc >= mmin && frame_fits(Mc, p->dx, p->dy, p->cx, p->cy, rxy, vlo, vhi)) {
            p->M = Mc;
            break;
        }
    }
    if (!p->M) return bail(fail(NURSD_ERR_GEOMETRY, "no supported transform size fits the geometry"));
    for (int a = 0; a < 2; ++a) {
        p->vlo[a] = vlo[a];
        p->vhi[a] = vhi[a];
    }
    p->Mf = 2 * p->M;
    p->BS = (p->M / 2 + 1 + 7) / 8 * 8;
    if (p->scaled()) {
        if (p->nx != p->ny) return bail(fail(NURSD_ERR_UNSUPPORTED_SIZE, "SRSD needs a square grid (nx == ny)"));
        if (p->M < 512) return bail(fail(NURSD_ERR_UNSUPPORTED_SIZE, "SRSD needs a transform size M >= 512"));
    }
    if (p->has_lists()) {
        if (p->M < 512)
            return bail(fail(NURSD_ERR_UNSUPPORTED_SIZE, "voxel lists need a transform size M >= 512 (set options.M)"));
        // fine rows each plane's interpolation can reach (centred fine cells;
        // a scaled plane has pitch dy / alpha)
        std::vector<int> lo(p->nz), hi(p->nz);
        const double hw = 0.5 * p->w;
        const int MF = p->Mf, RB = kType2RowBand;
        if (p->w > RB) return bail(fail(NURSD_ERR_ARG, "kernel width above the interpolation band"));
        auto first_row = [&](int v, double pitch) {
            const double t = ((double)vxy[2 * v + 1] - p->cy) / pitch * 2.0 + MF / 2;
            return (int)std::ceil(t - hw);
        };
        // interpolation entries: a voxel's w rows fall in one or two bands of
        // RB rows counted from the plane's first reachable row; one entry per
        // (voxel, band), sorted by plane, band and voxel
        std::vector<int> pband(p->nz + 1, 0), bptr(1, 0), evox, vent((size_t)p->nvox() * 2, -1);
        for (int iz = 0; iz < p->nz; ++iz) {
            const double pitch = p->mode == NURSD_MODE_SRSD_POINTS ? p->dy / p->alpha[iz] : p->dy;
            int a = 1 << 30, c = -(1 << 30);
            for (int v = p->plane_ptr[iz]; v < p->plane_ptr[iz + 1]; ++v) {
                const int i0 = first_row(v, pitch);
                a = std::min(a, i0);
                c = std::max(c, i0 + p->w - 1);
            }
            if (a > c) {          // empty plane
                a = 0;
                c = -1;
            } else if (c - a + 1 >= MF) {
                a = 0;
                c = MF - 1;
            }
            lo[iz] = a;
            hi[iz] = c;
            const int nb = c >= a ? (c - a) / RB + 1 : 0;
            pband[iz + 1] = pband[iz] + nb;
            std::vector<std::vector<int>> lists(nb);
            for (int v = p->plane_ptr[iz]; v < p->plane_ptr[iz + 1]; ++v) {
                const int i0 = first_row(v, pitch);
                const int b0 = ((i0 - a) & (MF - 1)) / RB, b1 = ((i0 + p->w - 1 - a) & (MF - 1)) / RB;
                lists[b0].push_back(v);
                if (b1 != b0) lists[b1].push_back(v);
            }
            for (int b = 0; b < nb; ++b) {
                for (int v : lists[b]) {
                    int* ve = &vent[2 * (size_t)v];
                    ve[ve[0] < 0 ? 0 : 1] = (int)evox.size();
                    evox.push_back(v);
                }
                bptr.push_back((int)evox.size());
            }
            p->max_vox = std::max(p->max_vox, p->plane_ptr[iz + 1] - p->plane_ptr[iz]);
        }
        p->n_lent = (int)evox.size();
        if ((rc = upload(p, lo, &p->d_row_lo))) return bail(rc);
        if ((rc = upload(p, hi, &p->d_row_hi))) return bail(rc);
        if ((rc = upload(p, pband, &p->d_plane_band))) return bail(rc);
        if ((rc = upload(p, bptr, &p->d_lband_ptr))) return bail(rc);
        if ((rc = upload(p, evox, &p->d_ent_vox))) return bail(rc);
        if ((rc = upload(p, vent, &p->d_vox_ent))) return bail(rc);
        if ((rc = upload(p, p->plane_ptr, &p->d_plane_ptr))) return bail(rc);
    }

    if (p->mode == NURSD_MODE_GRID3D) {
        // relays on a non-planar surface: depths, the intermediate plane and
        // the depth grid of stage 1
        if (!geo->relay_z_dev) return bail(fail(NURSD_ERR_ARG, "GRID3D mode needs relay_z_dev"));
        std::vector<float> rz;
        if ((rc = read_points(geo->relay_z_dev, (size_t)p->L, rz, s))) return bail(rc);
        p->z_mid = geo->z_mid;
        if (!std::isfinite(p->z_mid)) return bail(fail(NURSD_ERR_GEOMETRY, "non-finite z_mid"));
        for (double zz : p->z)
            if (!(zz > p->z_mid)) return bail(fail(NURSD_ERR_GEOMETRY, "voxel planes must lie beyond z_mid"));
        p->dz3 = geo->dz3 > 0 ? geo->dz3 : p->vdx;
        double ext = 0;
        for (float v : rz) {
            if (!std::isfinite(v)) return bail(fail(NURSD_ERR_GEOMETRY, "non-finite relay depth"));
            ext = std::max(ext, std::fabs((double)v - p->z_mid));
        }
        if (geo->mz3 > 0) {
            if (!is_pow2(geo->mz3) || geo->mz3 < 2 || geo->mz3 > 64)
                return bail(fail(NURSD_ERR_UNSUPPORTED_SIZE, "mz3 must be a power of two in [2, 64]"));
            p->Mz3 = geo->mz3;
            if (!(ext < 0.5 * p->Mz3 * p->dz3))
                return bail(fail(NURSD_ERR_GEOMETRY, "relay depths outside the depth period of the 3D grid"));
        } else {
            for (int m = 8; m <= 64 && !p->Mz3; m *= 2)
                if (ext <= 0.25 * m * p->dz3) p->Mz3 = m;
            if (!p->Mz3) return bail(fail(NURSD_ERR_GEOMETRY, "relay depths span more than 16 depth pitches"));
        }
        const int Mz = p->Mz3;
        // W_p(l) = Mz^-1 sum_{kz in I_Mz} e^{-j kz (z~_l + 2 pi p / Mz)}, p in I_Mz
        std::vector<float2> W((size_t)Mz * p->L);
        for (int l = 0; l < p->L; ++l) {
            const double zt = 2.0 * M_PI * ((double)rz[l] - p->z_mid) / (Mz * p->dz3);
            for (int pi = 0; pi < Mz; ++pi) {
                const double th = zt + 2.0 * M_PI * (pi - Mz / 2) / Mz;
                double re = 0, im = 0;
                for (int kz = -Mz / 2; kz < Mz / 2; ++kz) {
                    re += std::cos(kz * th);
                    im -= std::sin(kz * th);
                }
                W[(size_t)pi * p->L + l] = make_float2((float)(re / Mz), (float)(im / Mz));
            }
        }
        std::vector<double> zk(Mz);
        for (int pi = 0; pi < Mz; ++pi) zk[pi] = std::fabs((double)(pi - Mz / 2)) * p->dz3;
        if ((rc = upload(p, W, &p->d_W3))) return bail(rc);
        if ((rc = upload(p, zk, &p->d_zk3))) return bail(rc);
        p->FZ3 = std::max(1, std::min(p->F, 128 / Mz));
        // stage 2 propagates from z_mid: kernel distances z - z_mid, and the
        // illumination distance keeps the true depth
        for (double& zz : p->z) zz -= p->z_mid;
        p->xp[2] -= p->z_mid;
    }

    // chunking: about 128 planes of 512^2 per propagation chunk
    const long target = std::max(16L, std::min(4096L, 128L * (512L * 512L) / ((long)p->M * p->M)));
    p->FC = opt->freq_chunk > 0 ? opt->freq_chunk : std::min(p->F, 8);
    p->FC = std::min(p->FC, p->F);
    // the propagation kernels step phases from one frequency to the next by a
    // fixed factor: uneven bin lists run one frequency per chunk
    if (!even_bins(p)) p->FC = 1;
    p->ZC = opt->plane_chunk > 0 ? opt->plane_chunk : (int)std::max(1L, target / p->FC);
    if (p->has_lists() && opt->plane_chunk <= 0) p->ZC = std::max(1, 32 / p->FC);
    p->ZC = std::min(p->ZC, p->nz);
    // frequencies (3D: frequency-depth pairs) per spreading launch
    p->FCn = std::min(p->mode == NURSD_MODE_GRID3D ? p->F * p->Mz3 : p->F, 32);

    // device tables
    {
        std::vector<float2> tw;
        for (int n = 0; n < kMaxLog; ++n) {
            p->tw_off[n] = tw.size();
            const int N = 1 << n;
            for (int m = 0; m < N; ++m) {
                const double a = -2.0 * M_PI * (double)m / N;
                tw.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
            }
        }
        if ((rc = upload(p, tw, &p->tw_all))) return bail(rc);
    }
    {
        std::vector<float2> wt, tb;
        const double sf = p->sigma_rel * fc;
        for (int j = 0; j < p->F; ++j) {
            const double f = p->freqs[j];
            const double g = std::exp(-(f - fc) * (f - fc) / (2.0 * sf * sf));
            const double ph = -2.0 * M_PI * std::fmod(f * p->t0, 1.0);
            wt.push_back(make_float2((float)(g * std::cos(ph)), (float)(g * std::sin(ph))));
            const double a = -2.0 * M_PI * (double)p->bins[j] / p->T;
            tb.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
        }
        if ((rc = upload(p, p->bins, &p->d_bins))) return bail(rc);
        if ((rc = upload(p, wt, &p->d_wt))) return bail(rc);
        if ((rc = upload(p, tb, &p->d_tb))) return bail(rc);
        if ((rc = upload(p, p->freqs, &p->d_f))) return bail(rc);
        if ((rc = upload(p, p->z, &p->d_z))) return bail(rc);
        if (p->scaled()) {
            std::vector<double> px, py;
            for (double a : p->alpha) {
                px.push_back(p->dx / a);
                py.push_back(p->dy / a);
            }
            if ((rc = upload(p, px, &p->d_px))) return bail(rc);
            if ((rc = upload(p, py, &p->d_py))) return bail(rc);
            if ((rc = upload(p, p->alpha, &p->d_alpha))) return bail(rc);
            // Bluestein chirp h'[j] = e^{+j pi alpha (j - D)^2 / M}, D = M/2 - N/2.
            // The M outputs of a scaled line come in two halves k' in
            // [k0, k0 + M/2), k0 = 0, M/2; half k0 is the circular convolution
            // of length M of the pre-chirped input (n in [0, N)) with
            // h'[k0 + j], j in [-(N-1), M/2 - 1] at j mod M, exact while
            // N + M/2 - 1 <= M.  Spectra stored [Z][2][M], divided by M (inverse
            // FFT of the convolution) and by M (each of the two passes carries
            // one factor of the M^-2 of the final inverse transform).
            const int M = p->M, N = p->nx, D = M / 2 - N / 2;
            if (N + M / 2 - 1 > M)
                return bail(fail(NURSD_ERR_UNSUPPORTED_SIZE, "scaled RSD needs M >= 2 (N - 1) (pad >= 2)"));
            std::vector<float2> hh((size_t)p->nz * 2 * M);
            std::vector<std::complex<double>> line(M);
            for (int iz = 0; iz < p->nz; ++iz)
                for (int half = 0; half < 2; ++half) {
                    const int k0 = half * (M / 2);
                    std::fill(line.begin(), line.end(), std::complex<double>(0, 0));
                    for (int j = -(N - 1); j <= M / 2 - 1; ++j) {
                        const double dd = (double)(k0 + j - D);
                        const double cyc = std::fmod(p->alpha[iz] * dd * dd / (2.0 * M), 1.0);
                        line[(j + M) % M] = std::polar(1.0, 2.0 * M_PI * cyc);
                    }
                    fft64(line);
                    for (int k = 0; k < M; ++k)
                        hh[((size_t)iz * 2 + half) * M + k] =
                            make_float2((float)(line[k].real() / ((double)M * M)), (float)(line[k].imag() / ((double)M * M)));
                }
            if ((rc = upload(p, hh, &p->d_hhat))) return bail(rc);
            // the chirp itself, c[j] = e^{-j pi alpha m^2 / M} at m = j - M/2
            std::vector<float2> cz((size_t)p->nz * M);
            for (int iz = 0; iz < p->nz; ++iz)
                for (int j = 0; j < M; ++j) {
                    const double m = (double)(j - M / 2);
                    const double cyc = std::fmod(p->alpha[iz] * m * m / (2.0 * M), 1.0);
                    cz[(size_t)iz * M + j] = make_float2((float)std::cos(2.0 * M_PI * cyc),
                                                         (float)-std::sin(2.0 * M_PI * cyc));
                }
            if ((rc = upload(p, cz, &p->d_chirp))) return bail(rc);
        }
    }
    {
        // deconvolution: phihat(k) = (w/2) int_{-1}^{1} psi(z) cos(pi k w z / Mf) dz
        std::vector<double> gx, gw;
        gauss_legendre(128, gx, gw);
        std::vector<float> decx(p->M), decy(p->M);
        for (int km = 0; km < p->M; ++km) {
            const int k = km < p->M / 2 ? km : km - p->M;
            double s = 0;
            for (size_t q = 0; q < gx.size(); ++q)
                s += gw[q] * es_psi(gx[q], p->beta) * std::cos(kPi * k * p->w * gx[q] / p->Mf);
            const double ph = 0.5 * p->w * s;
            const double sgn = (k & 1) ? -1.0 : 1.0;
            decy[km] = (float)(sgn / ph);
            decx[km] = (float)(sgn / (ph * (double)p->M * p->M));
        }
        if ((rc = upload(p, decx, &p->d_decx))) return bail(rc);
        if ((rc = upload(p, decy, &p->d_decy))) return bail(rc);
    }
    if (opt->weights_dev) {
        std::vector<float> wv;
        if ((rc = read_points(opt->weights_dev, (size_t)p->L, wv, s))) return bail(rc);
        for (float v : wv)
            if (!std::isfinite(v)) return bail(fail(NURSD_ERR_ARG, "non-finite sample weight"));
        if ((rc = upload(p, wv, &p->d_w))) return bail(rc);
    }
    if (opt->spread_tile) {
        if (!spread_var_plain_ok(p->Mf, opt->spread_tile))
            return bail(fail(NURSD_ERR_ARG, "spreading tile " + std::to_string(opt->spread_tile) +
                                                 " is not available for a fine grid of " + std::to_string(p->Mf)));
        p->spread_var = opt->spread_tile;
    } else {
        p->spread_var = p->mode == NURSD_MODE_GRID3D ? NURSD_PLAN3D_SPREAD_VAR : NURSD_PLAN_SPREAD_VAR;
        if (!spread_var_plain_ok(p->Mf, p->spread_var)) p->spread_var = 0;
    }
    if ((rc = build_spread_lists(p, rxy))) return bail(rc);
    layout_workspace(p);
    // device address of the fixed scratch of nursd_forward_hist_static on
    // this device (looked up once per device)
    void* scr = nullptr;
    if ((rc = static_scratch(&scr))) return bail(rc);
    *out = p;
    return NURSD_OK;
}

static int nursd_plan_set_points_body(nursd_plan* p, const float* relay_xy_dev, void* stream) {
    if (!p || !relay_xy_dev) return fail(NURSD_ERR_ARG, "NULL argument");
    std::vector<float> rxy;
    int rc = read_points(relay_xy_dev, (size_t)p->L * 2, rxy, static_cast<hipStream_t>(stream));
    if (rc) return rc;
    for (float v : rxy)
        if (!std::isfinite(v)) return fail(NURSD_ERR_GEOMETRY, "non-finite relay position");
    // the frame rule of plan creation: relays inside the period and every
    // relay-voxel offset inside half a period (else the circular convolution
    // would wrap)
    if (!frame_fits(p->M, p->dx, p->dy, p->cx, p->cy, rxy, p->vlo, p->vhi))
        return fail(NURSD_ERR_GEOMETRY, "relay positions leave the plan's frame (period or half-period offset rule)");
    return build_spread_lists(p, rxy);
}

int nursd_plan_info(const nursd_plan* p, nursd_plan_info_t* info) {
    if (!p || !info) return fail(NURSD_ERR_ARG, "NULL argument");
    info->M = p->M;
    info->Mf = p->Mf;
    info->n_freq = p->F;
    info->n_relay = p->L;
    info->kernel_width = p->w;
    info->n_voxels = p->nvox();
    info->dx = p->dx;
    info->dy = p->dy;
    info->cx = p->cx;
    info->cy = p->cy;
    info->beta = p->beta;
    info->workspace_bytes = p->ws_bytes;
    info->freq_chunk = p->FC;
    info->plane_chunk = p->ZC;
    info->depth3d = p->Mz3;
    info->upsample_q = p->q;
    return NURSD_OK;
}

int nursd_workspace_size(const nursd_plan* p, size_t* bytes) {
    if (!p || !bytes) return fail(NURSD_ERR_ARG, "NULL argument");
    *bytes = p->ws_bytes;
    return NURSD_OK;
}

void nursd_plan_destroy(nursd_plan* p) { delete p; }

int nursd_phasor(nursd_plan* p, const float* hist, void* P, void* stream) {
    if (!p || !hist || !P) return fail(NURSD_ERR_ARG, "NULL argument");
    if (reinterpret_cast<uintptr_t>(hist) & 7) return fail(NURSD_ERR_ARG, "histograms must be 8-byte aligned");
    if (!is_pow2(p->T) || p->T < 256 || p->T > 8192)
        return fail(NURSD_ERR_UNSUPPORTED_SIZE, "T must be a power of two in [256, 8192]");
    PhasorArgs a{};
    a.hist = hist;
    a.P = static_cast<float2*>(P);
    a.L = p->L;
    a.T = p->T;
    a.F = p->F;
    a.bins = p->d_bins;
    a.wt = p->d_wt;
    a.tb = p->d_tb;
    a.tw = p->tw(p->T / 2);
    LAUNCH(p, NURSD_STAGE_PHASOR, PhasorArgs, launch_phasor, a, static_cast<hipStream_t>(stream));
    return NURSD_OK;
}

int nursd_spectrum(nursd_plan* p, const void* P, void* U, void* ws, size_t ws_bytes, void* stream) {
    if (!p || !P || !U) return fail(NURSD_ERR_ARG, "NULL argument");
    int rc = check_ws(p, ws, ws_bytes);
    if (rc) return rc;
    return run_spectrum(p, static_cast<const float2*>(P), static_cast<float2*>(U), static_cast<char*>(ws),
                        static_cast<hipStream_t>(stream));
}

int nursd_forward_phasor(nursd_plan* p, const void* P, void* vol, float* I, void* ws, size_t ws_bytes,
                         void* stream) {
    if (!p || !P) return fail(NURSD_ERR_ARG, "NULL argument");
    if (!vol && !I) return fail(NURSD_ERR_ARG, "vol and I are both NULL");
    if (!p->coherent && vol) return fail(NURSD_ERR_ARG, "incoherent plans produce intensity only");
    int rc = check_ws(p, ws, ws_bytes);
    if (rc) return rc;
    return forward_from_P(p, static_cast<const float2*>(P), vol, I, static_cast<char*>(ws),
                          static_cast<hipStream_t>(stream));
}

int nursd_forward_hist(nursd_plan* p, const float* hist, void* vol, float* I, void* ws, size_t ws_bytes,
                       void* stream) {
    if (!p || !hist) return fail(NURSD_ERR_ARG, "NULL argument");
    if (!vol && !I) return fail(NURSD_ERR_ARG, "vol and I are both NULL");
    if (!p->coherent && vol) return fail(NURSD_ERR_ARG, "incoherent plans produce intensity only");
    int rc = check_ws(p, ws, ws_bytes);
    if (rc) return rc;
    char* w = static_cast<char*>(ws);
    float2* P = reinterpret_cast<float2*>(w + p->off_P);
    if ((rc = nursd_phasor(p, hist, P, stream))) return rc;
    return forward_from_P(p, P, vol, I, w, static_cast<hipStream_t>(stream));
}

int nursd_forward_hist_static(nursd_plan* p, const float* hist, void* vol, float* I, void* stream) {
    if (!p || !hist) return fail(NURSD_ERR_ARG, "NULL argument");
    if (p->ws_bytes > kStaticScratchBytes)
        return fail(NURSD_ERR_WORKSPACE, "plan needs " + std::to_string(p->ws_bytes) +
                                             " bytes of workspace; the fixed scratch holds " +
                                             std::to_string(kStaticScratchBytes) +
                                             " (use nursd_forward_hist with a caller workspace)");
    if (p->prof_mask) return fail(NURSD_ERR_ARG, "profiling creates events; end it before this call");
    void* scr = nullptr;
    int rc = static_scratch(&scr);
    if (rc) return rc;
    return nursd_forward_hist(p, hist, vol, I, scr, kStaticScratchBytes, stream);
}

namespace {

bool video_ok(const nursd_plan* p) {
    return p->coherent && (p->mode == NURSD_MODE_GRID || p->mode == NURSD_MODE_SRSD);
}
size_t video_field_bytes(const nursd_plan* p) {
    return align_up((size_t)p->F * p->ZC * p->nx * p->ny * sizeof(float2));
}

}  // namespace

int nursd_video_workspace_size(const nursd_plan* p, size_t* bytes) {
    if (!p || !bytes) return fail(NURSD_ERR_ARG, "NULL argument");
    if (!video_ok(p)) return fail(NURSD_ERR_UNSUPPORTED_SIZE, "video needs a coherent GRID or SRSD plan");
    *bytes = p->ws_bytes + video_field_bytes(p);
    return NURSD_OK;
}

int nursd_forward_video(nursd_plan* p, const void* P, int32_t n_frames, double t_first, double t_step,
                        void* video, float* video_I, void* ws, size_t ws_bytes, void* stream) {
    if (!p || !P) return fail(NURSD_ERR_ARG, "NULL argument");
    if (!video && !video_I) return fail(NURSD_ERR_ARG, "video and video_I are both NULL");
    if (n_frames < 1) return fail(NURSD_ERR_ARG, "n_frames must be >= 1");
    if (!std::isfinite(t_first) || !std::isfinite(t_step)) return fail(NURSD_ERR_ARG, "non-finite time");
    if (!video_ok(p)) return fail(NURSD_ERR_UNSUPPORTED_SIZE, "video needs a coherent GRID or SRSD plan");
    int rc = check_ws(p, ws, ws_bytes);
    if (rc) return rc;
    if (ws_bytes < p->ws_bytes + video_field_bytes(p))
        return fail(NURSD_ERR_WORKSPACE, "workspace too small for the video: need " +
                                             std::to_string(p->ws_bytes + video_field_bytes(p)) + " bytes");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    float2* field = reinterpret_cast<float2*>(w + p->ws_bytes);
    float2* U = reinterpret_cast<float2*>(w + p->off_U);
    if ((rc = run_spectrum(p, static_cast<const float2*>(P), U, w, s))) return rc;
    float2* Bt = reinterpret_cast<float2*>(w + p->off_Bt);
    float2* Yt = reinterpret_cast<float2*>(w + p->off_Yt);
    float2* u = reinterpret_cast<float2*>(w + p->off_u);
    const bool scaled = p->mode == NURSD_MODE_SRSD;
    if (scaled) {
        RelayGridArgs ra{};
        ra.U = U;
        ra.Tg = reinterpret_cast<float2*>(w + p->off_Tg);
        ra.u = u;
        ra.M = p->M;
        ra.N = p->nx;
        ra.b0 = 0;
        ra.nb = p->F;
        ra.tw_m = p->tw(p->M);
        LAUNCH(p, NURSD_STAGE_RELAY_GRID, RelayGridArgs, launch_relay_grid, ra, s);
    }
    // slab by slab: every frequency's field for ZC planes, then the frames
    for (int z0 = 0; z0 < p->nz; z0 += p->ZC) {
        const int nzc = std::min(p->ZC, p->nz - z0);
        for (int b0 = 0; b0 < p->F; b0 += p->FC) {
            const int nb = std::min(p->FC, p->F - b0);
            const ChunkGeom g = chunk_geom(p, b0, nb, z0, nzc);
            P1Args a1 = kernel_args(p, g, Bt);
            LAUNCH(p, NURSD_STAGE_KERNEL_ROWS, P1Args, launch_kernel_rows, a1, s);
            if (scaled) {
                ChirpArgs ca{};
                ca.g = g;
                ca.u = u;
                ca.S1t = reinterpret_cast<float2*>(w + p->off_S1);
                ca.Bt = Bt;
                ca.Yt = Yt;
                ca.M = p->M;
                ca.N = p->nx;
                ca.BS = p->BS;
                ca.ny = p->ny;
                ca.alpha = p->d_alpha;
                ca.hhat = p->d_hhat;
                ca.chirp = p->d_chirp;
                ca.tw_m = p->tw(p->M);
                ca.tw_lb = p->tw(2 * p->M);
                LAUNCH(p, NURSD_STAGE_CHIRP_ROWS, ChirpArgs, launch_chirp_rows, ca, s);
                LAUNCH(p, NURSD_STAGE_PROPAGATE_COLS, ChirpArgs, launch_chirp_cols, ca, s);
            } else {
                P2Args a2 = cols_args(p, g, Bt, U, Yt);
                LAUNCH(p, NURSD_STAGE_PROPAGATE_COLS, P2Args, launch_propagate_cols, a2, s);
            }
            P3Args a3 = rows_args(p, g, Yt, nullptr, nullptr, b0, nb);
            a3.first = 1;
            a3.field = field;
            a3.field_z0 = z0;
            a3.field_nz = p->ZC;
            LAUNCH(p, NURSD_STAGE_PROPAGATE_ROWS, P3Args, launch_propagate_rows, a3, s);
        }
        VideoArgs va{};
        va.field = field;
        va.f = p->d_f;
        va.V = static_cast<float2*>(video);
        va.I = video_I;
        va.F = p->F;
        va.field_nz = p->ZC;
        va.nzc = nzc;
        va.z0 = z0;
        va.nz = p->nz;
        va.nvp = p->nx * p->ny;
        va.T = n_frames;
        va.t_first = t_first;
        va.t_step = t_step;
        LAUNCH(p, NURSD_STAGE_VIDEO, VideoArgs, launch_video, va, s);
    }
    return NURSD_OK;
}

namespace {

size_t multi_spectra_bytes(const nursd_plan* p, int K) {
    return align_up((size_t)K * p->F * p->M * p->M * sizeof(float2));
}

}  // namespace

int nursd_multi_workspace_size(const nursd_plan* p, int32_t K, size_t* bytes) {
    if (!p || !bytes) return fail(NURSD_ERR_ARG, "NULL argument");
    if (K < 1) return fail(NURSD_ERR_ARG, "K must be >= 1");
    if (p->mode != NURSD_MODE_GRID || !p->coherent)
        return fail(NURSD_ERR_UNSUPPORTED_SIZE, "several illumination positions need a coherent GRID plan");
    *bytes = p->ws_bytes + multi_spectra_bytes(p, K);
    return NURSD_OK;
}

int nursd_forward_multi(nursd_plan* p, const void* P, int32_t K, const double* xp, void* vol, float* I, void* ws,
                        size_t ws_bytes, void* stream) {
    if (!p || !P || !xp) return fail(NURSD_ERR_ARG, "NULL argument");
    if (!vol && !I) return fail(NURSD_ERR_ARG, "vol and I are both NULL");
    if (K < 1) return fail(NURSD_ERR_ARG, "K must be >= 1");
    if (p->mode != NURSD_MODE_GRID || !p->coherent)
        return fail(NURSD_ERR_UNSUPPORTED_SIZE, "several illumination positions need a coherent GRID plan");
    for (int i = 0; i < 3 * K; ++i)
        if (!std::isfinite(xp[i])) return fail(NURSD_ERR_GEOMETRY, "non-finite illumination position");
    int rc = check_ws(p, ws, ws_bytes);
    if (rc) return rc;
    if (ws_bytes < p->ws_bytes + multi_spectra_bytes(p, K))
        return fail(NURSD_ERR_WORKSPACE, "workspace too small for K positions: need " +
                                             std::to_string(p->ws_bytes + multi_spectra_bytes(p, K)) + " bytes");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    const size_t uk = (size_t)p->F * p->M * p->M;
    float2* Us = reinterpret_cast<float2*>(w + p->ws_bytes);
    for (int k = 0; k < K; ++k)
        if ((rc = run_spectrum(p, static_cast<const float2*>(P) + (size_t)k * p->F * p->L, Us + k * uk, w, s)))
            return rc;
    float2* V = vol ? static_cast<float2*>(vol) : reinterpret_cast<float2*>(w + p->off_V);
    float2* Bt = reinterpret_cast<float2*>(w + p->off_Bt);
    float2* Yt = reinterpret_cast<float2*>(w + p->off_Yt);
    for (int b0 = 0; b0 < p->F; b0 += p->FC) {
        const int nb = std::min(p->FC, p->F - b0);
        for (int z0 = 0; z0 < p->nz; z0 += p->ZC) {
            const int nzc = std::min(p->ZC, p->nz - z0);
            const ChunkGeom g = chunk_geom(p, b0, nb, z0, nzc);
            P1Args a1 = kernel_args(p, g, Bt);
            LAUNCH(p, NURSD_STAGE_KERNEL_ROWS, P1Args, launch_kernel_rows, a1, s);
            for (int k = 0; k < K; ++k) {       // the kernel spectrum serves every position
                P2Args a2 = cols_args(p, g, Bt, Us + k * uk, Yt);
                LAUNCH(p, NURSD_STAGE_PROPAGATE_COLS, P2Args, launch_propagate_cols, a2, s);
                P3Args a3 = rows_args(p, g, Yt, V, I, b0, nb);
                a3.xp0 = xp[3 * k];
                a3.xp1 = xp[3 * k + 1];
                a3.xp2 = xp[3 * k + 2];
                a3.first = b0 == 0 && k == 0;
                a3.last = b0 + nb >= p->F && k == K - 1;
                LAUNCH(p, NURSD_STAGE_PROPAGATE_ROWS, P3Args, launch_propagate_rows, a3, s);
            }
        }
    }
    return NURSD_OK;
}

int nursd_subsample_nearest(const void* in, void* out, int32_t F, int32_t ny, int32_t nx, int32_t D, void* stream) {
    if (!in || !out) return fail(NURSD_ERR_ARG, "NULL argument");
    if (in == out) return fail(NURSD_ERR_ARG, "in and out must be different buffers");
    if (F < 1 || ny < 1 || nx < 1 || D < 1) return fail(NURSD_ERR_ARG, "F, ny, nx and D must be >= 1");
    HIP_TRY(launch_subsample_nearest(static_cast<const float2*>(in), static_cast<float2*>(out), F, ny, nx, D,
                                     static_cast<hipStream_t>(stream)));
    return NURSD_OK;
}

int nursd_adjoint(nursd_plan* p, const void* grad_vol, const void* P, void* grad_P, float* grad_xy, void* ws,
                  size_t ws_bytes, void* stream) {
    if (!p || !grad_vol || !grad_P) return fail(NURSD_ERR_ARG, "NULL argument");
    if (grad_xy && !P) return fail(NURSD_ERR_ARG, "the position gradient needs P");
    if (p->mode != NURSD_MODE_GRID || !p->coherent)
        return fail(NURSD_ERR_UNSUPPORTED_SIZE, "the adjoint is defined for coherent GRID plans");
    int rc = check_ws(p, ws, ws_bytes);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    AdjArgs a{};
    a.gV = static_cast<const float2*>(grad_vol);
    a.Rt = reinterpret_cast<float2*>(w + p->off_Yt);
    a.Bt = reinterpret_cast<float2*>(w + p->off_Bt);
    a.St = reinterpret_cast<float2*>(w + p->off_U);
    a.T3 = reinterpret_cast<float2*>(w + p->off_T3);
    a.G3 = reinterpret_cast<float2*>(w + p->off_G3);
    a.P = static_cast<const float2*>(P);
    a.grad_P = static_cast<float2*>(grad_P);
    a.grad_xy = grad_xy;
    a.relay = p->d_relay;
    a.tw_m = p->tw(p->M);
    a.tw_f = p->tw(p->Mf);
    a.dec = p->d_decy;
    a.M = p->M;
    a.Mf = p->Mf;
    a.BS = p->BS;
    a.nx = p->nx;
    a.ny = p->ny;
    a.L = p->L;
    a.w = p->w;
    a.beta = (float)p->beta;
    a.kscale_x = (float)(2.0 * M_PI / (p->M * p->dx));
    a.kscale_y = (float)(2.0 * M_PI / (p->M * p->dy));
    a.xc = p->cx;
    a.yc = p->cy;
    a.cx = p->cx;
    a.cy = p->cy;
    a.xp0 = p->xp[0];
    a.xp1 = p->xp[1];
    a.xp2 = p->xp[2];
    a.relay_row_lo = p->relay_row_lo;
    a.relay_row_hi = p->relay_row_hi;
    a.q = p->q;
    a.wts = p->d_w;
    float2* Bt = const_cast<float2*>(a.Bt);
    for (int b0 = 0; b0 < p->F; b0 += p->FC) {
        const int nb = std::min(p->FC, p->F - b0);
        for (int z0 = 0; z0 < p->nz; z0 += p->ZC) {
            const int nzc = std::min(p->ZC, p->nz - z0);
            const ChunkGeom g = chunk_geom(p, b0, nb, z0, nzc);
            P1Args a1 = kernel_args(p, g, Bt);
            LAUNCH(p, NURSD_STAGE_KERNEL_ROWS, P1Args, launch_kernel_rows, a1, s);
            a.g = g;
            a.first = z0 == 0;
            LAUNCH(p, NURSD_STAGE_ADJOINT, AdjArgs, launch_adjoint_planes, a, s);
        }
    }
    for (int b0 = 0; b0 < p->F; b0 += p->FC3) {
        const int nb = std::min(p->FC3, p->F - b0);
        a.g = chunk_geom(p, b0, nb, 0, 1);
        a.first_b = b0 == 0;
        LAUNCH(p, NURSD_STAGE_TYPE2, AdjArgs, launch_adjoint_type2, a, s);
    }
    return NURSD_OK;
}

static int nursd_batch_create_body(nursd_plan* const* plans, int32_t n, int32_t autotune, void* stream, nursd_batch** out) {
    (void)stream;
    if (!out) return fail(NURSD_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!plans || n < 1) return fail(NURSD_ERR_ARG, "no plans");
    for (int i = 0; i < n; ++i) {
        if (!plans[i]) return fail(NURSD_ERR_ARG, "NULL plan");
        if (plans[i]->mode != NURSD_MODE_GRID || !plans[i]->coherent)
            return fail(NURSD_ERR_UNSUPPORTED_SIZE, "batched mode takes coherent GRID plans");
        if (!is_pow2(plans[i]->T) || plans[i]->T < 256 || plans[i]->T > 8192)
            return fail(NURSD_ERR_UNSUPPORTED_SIZE, "T must be a power of two in [256, 8192]");
        if (!even_bins(plans[i]))
            return fail(NURSD_ERR_UNSUPPORTED_SIZE, "batched mode needs evenly spaced frequency bins");
    }
    auto bt = new nursd_batch();
    auto bail = [&](int rc) {
        delete bt;
        return rc;
    };
    for (int i = 0; i < n; ++i) {
        BatchScene sc;
        sc.p = plans[i];
        bt->sc.push_back(sc);
    }
    bt->autotune = autotune ? 1 : 0;
    bt->hist.assign(n, nullptr);
    bt->I.assign(n, nullptr);
    if (int rc = batch_kernel_classes(bt)) return bail(rc);
    // Relay lists for the other spreading band heights the tuner may try, or
    // (without tuning) for the tile of the first plan of the size class when
    // a plan's own tile differs.
    bt->lists.assign(n, {});
    {
        for (int i = 0; i < n; ++i) {
            const nursd_plan* p = plans[i];
            const int class_br = spread_var_rows(batch_choice(bt, BK_SPREAD, p->Mf), p->Mf);
            for (int br : {1, 2, 4, 8, 16}) {
                if (br == spread_var_rows(p->spread_var, p->Mf) || p->Mf / br < 2) continue;
                if (!bt->autotune && br != class_br) continue;
                SpreadLists sl;
                if (int rc = bin_relays(p, p->h_relay, br, sl)) return bail(rc);
                BatchLists bl;
                bl.nbands = sl.nbands;
                auto put = [&](const void* src, size_t bytes, void** dst) -> int {
                    HIP_TRY(hipMalloc(dst, std::max<size_t>(bytes, 16)));
                    bt->owned.push_back(*dst);
                    if (bytes) HIP_TRY(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
                    return NURSD_OK;
                };
                void *d0 = nullptr, *d1 = nullptr, *d2 = nullptr;
                int rc = put(sl.ent.data(), sl.ent.size() * sizeof(SpreadEntry), &d0);
                if (!rc) rc = put(sl.band_ptr.data(), sl.band_ptr.size() * sizeof(int), &d1);
                if (!rc) rc = put(sl.wave_rng.data(), sl.wave_rng.size() * sizeof(int), &d2);
                if (rc) return bail(rc);
                bl.ent = static_cast<SpreadEntry*>(d0);
                bl.band_ptr = static_cast<int*>(d1);
                bl.wave_rng = static_cast<int*>(d2);
                bt->lists[i][br] = bl;
            }
        }
    }
    // Default configuration: work queue, scenes with M >= 512 chunk by chunk,
    // the fewest rounds whose propagation scratch fits the default budget.
    std::vector<int> rounds;
    for (int r : {4, 8, 16, 32, 64})
        if (batch_scratch_bytes(bt, r, 512) <= kBatchScratchCap) rounds.push_back(r);
    if (rounds.empty()) rounds.push_back(128);
    bt->cfg = BatchConfig{rounds.front(), kQueue, 512};
    for (int r : rounds)
        if (batch_scratch_bytes(bt, r, 512) <= kBatchScratchDefault) {
            bt->cfg.rounds = r;
            break;
        }
    // Tuner candidates: serial threshold x schedule x the two fewest rounds
    // whose grouped scratch fits the candidate limit.
    bt->cands.push_back(bt->cfg);
    if (bt->autotune) {
        bt->cands.clear();
        for (int mth : {256, 512, 1 << 20}) {
            std::vector<int> rs;
            for (int r : {4, 8, 16, 32, 64, 128})
                if (rs.size() < 2 && batch_scratch_bytes(bt, r, mth) <= kBatchScratchCap) rs.push_back(r);
            for (int sched : {kFlat, kQueue})
                for (int r : rs) bt->cands.push_back(BatchConfig{r, sched, mth});
        }
        if (bt->cands.empty()) bt->cands.push_back(bt->cfg);
    }
    // Size the workspace and the device tables for every candidate, with the
    // default schedule variants and (for the tuner) the finest ones.
    size_t tab_max = 0;
    int cnt_max = 0;
    for (int pass = 0; pass < (bt->autotune ? 2 : 1); ++pass) {
        if (pass == 1) finest_choices(bt);
        for (const BatchConfig& c : bt->cands) {
            bt->ws_need = std::max(bt->ws_need, batch_layout(bt, c));
            size_t tb = 0;
            int cn = 0;
            batch_table_size(bt, c, &tb, &cn);
            tab_max = std::max(tab_max, tb);
            cnt_max = std::max(cnt_max, cn);
        }
    }
    bt->choice.clear();
    bt->ws_need = std::max(bt->ws_need, batch_layout(bt, bt->cfg));
    if (bt->lists_missing) return bail(fail(NURSD_ERR_ARG, "batch spreading tile without binned relay lists"));
    bt->tab.clear();
    bt->launches.clear();
    hipError_t e;
    if (tab_max > 0) {
        void* d = nullptr;
        if ((e = hipMalloc(&d, tab_max)) != hipSuccess)
            return bail(fail(NURSD_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e)));
        bt->d_tab = static_cast<char*>(d);
        if ((e = hipHostMalloc(&bt->pinned, tab_max, hipHostMallocDefault)) != hipSuccess)
            return bail(fail(NURSD_ERR_HIP, std::string("hipHostMalloc: ") + hipGetErrorString(e)));
        bt->tab_cap = tab_max;
    }
    if (cnt_max > 0) {
        void* d = nullptr;
        if ((e = hipMalloc(&d, (size_t)cnt_max * sizeof(int))) != hipSuccess)
            return bail(fail(NURSD_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e)));
        bt->d_counters = static_cast<int*>(d);
        bt->counters_cap = cnt_max;
    }
    if ((e = hipEventCreateWithFlags(&bt->upload_done, hipEventDisableTiming)) != hipSuccess)
        return bail(fail(NURSD_ERR_HIP, std::string("hipEventCreate: ") + hipGetErrorString(e)));
    if ((e = hipStreamCreateWithFlags(&bt->cap, hipStreamNonBlocking)) != hipSuccess)
        return bail(fail(NURSD_ERR_HIP, std::string("hipStreamCreate: ") + hipGetErrorString(e)));
    *out = bt;
    return NURSD_OK;
}

int nursd_batch_workspace_size(const nursd_batch* bt, size_t* bytes) {
    if (!bt || !bytes) return fail(NURSD_ERR_ARG, "NULL argument");
    *bytes = bt->ws_need;
    return NURSD_OK;
}

static int nursd_batch_autotune_body(nursd_batch* bt, const float* const* hist, float* const* I, void* ws, size_t ws_bytes,
                         void* stream) {
    if (!bt) return fail(NURSD_ERR_ARG, "NULL batch");
    if (!bt->autotune) return fail(NURSD_ERR_ARG, "the batch was created without autotuning");
    hipStream_t s = static_cast<hipStream_t>(stream);
    bool changed = false;
    int rc = batch_check_io(bt, hist, I, ws, ws_bytes, &changed);
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = 1e30f;
    BatchConfig best_c = bt->cfg;
    bt->tried.clear();
    bt->tried_ms.clear();
    for (const BatchConfig& c : bt->cands) {
        bt->cfg = c;
        if ((rc = batch_bind(bt, static_cast<const char*>(ws), s))) break;
        hipError_t e = hipGraphLaunch(bt->exec, s);
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipGraphLaunch(bt->exec, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            rc = fail(NURSD_ERR_HIP, std::string("batch autotune: ") + hipGetErrorString(e));
            break;
        }
        bt->tried.push_back(config_code(c));
        bt->tried_ms.push_back(ms / 2);
        if (ms < best) {
            best = ms;
            best_c = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    bt->cfg = best_c;
    if (rc) {
        bt->ready = false;
        return rc;
    }
    if ((rc = batch_tune_kernels(bt, static_cast<const char*>(ws), s))) {
        bt->ready = false;
        return rc;
    }
    return batch_bind(bt, static_cast<const char*>(ws), s);
}

static int nursd_batch_forward_body(nursd_batch* bt, const float* const* hist, float* const* I, void* ws, size_t ws_bytes,
                        void* stream) {
    if (!bt) return fail(NURSD_ERR_ARG, "NULL batch");
    hipStream_t s = static_cast<hipStream_t>(stream);
    bool changed = false;
    int rc = batch_check_io(bt, hist, I, ws, ws_bytes, &changed);
    if (rc) return rc;
    if (changed && (rc = batch_bind(bt, static_cast<const char*>(ws), s))) return rc;
    HIP_TRY(hipGraphLaunch(bt->exec, s));
    return NURSD_OK;
}

int nursd_batch_info(const nursd_batch* bt, int32_t* budget, int32_t* launches, int32_t* n_tried, int32_t* tried,
                     float* tried_ms, size_t* workspace_bytes) {
    if (!bt) return fail(NURSD_ERR_ARG, "NULL batch");
    if (budget) *budget = config_code(bt->cfg);
    if (launches) *launches = (int32_t)bt->launches.size();
    if (n_tried) *n_tried = (int32_t)bt->tried.size();
    for (size_t i = 0; i < bt->tried.size() && i < 16; ++i) {
        if (tried) tried[i] = bt->tried[i];
        if (tried_ms) tried_ms[i] = bt->tried_ms[i];
    }
    if (workspace_bytes) *workspace_bytes = bt->ws_need;
    return NURSD_OK;
}

static int nursd_batch_tuning_body(const nursd_batch* bt, char* buf, size_t len) {
    if (!bt || !buf || len == 0) return fail(NURSD_ERR_ARG, "NULL argument");
    std::string t;
    for (size_t i = 0; i < bt->tuned.size(); ++i) t += (i ? "; " : "") + bt->tuned[i];
    std::snprintf(buf, len, "%s", t.c_str());
    return NURSD_OK;
}

void nursd_batch_destroy(nursd_batch* bt) { delete bt; }

int nursd_profile_begin(nursd_plan* p, uint32_t mask) {
    if (!p) return fail(NURSD_ERR_ARG, "NULL plan");
    p->prof_mask = mask;
    p->ev_used = 0;
    p->ev_stage.clear();
    return NURSD_OK;
}

int nursd_profile_end(nursd_plan* p, double* ms, int32_t* calls) {
    if (!p || !ms || !calls) return fail(NURSD_ERR_ARG, "NULL argument");
    for (int i = 0; i < NURSD_NUM_STAGES; ++i) {
        ms[i] = 0.0;
        calls[i] = 0;
    }
    for (size_t i = 0; i < p->ev_stage.size(); ++i) {
        HIP_TRY(hipEventSynchronize(p->ev_pool[2 * i + 1]));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, p->ev_pool[2 * i], p->ev_pool[2 * i + 1]));
        ms[p->ev_stage[i]] += t;
        calls[p->ev_stage[i]] += 1;
    }
    p->prof_mask = 0;
    p->ev_used = 0;
    p->ev_stage.clear();
    return NURSD_OK;
}

const char* nursd_last_error(void) { return g_err.c_str(); }


// Entry points whose bodies use host containers: no C++ exception crosses
// the C ABI.
int nursd_plan_create(const nursd_wavelet* wl, const nursd_geometry* geo, const nursd_options* opt,
                      const float* relay_xy_dev, void* stream, nursd_plan** out) {
    NURSD_GUARD(nursd_plan_create_body(wl, geo, opt, relay_xy_dev, stream, out));
}

int nursd_plan_set_points(nursd_plan* p, const float* relay_xy_dev, void* stream) {
    NURSD_GUARD(nursd_plan_set_points_body(p, relay_xy_dev, stream));
}

int nursd_batch_create(nursd_plan* const* plans, int32_t n, int32_t autotune, void* stream, nursd_batch** out) {
    NURSD_GUARD(nursd_batch_create_body(plans, n, autotune, stream, out));
}

int nursd_batch_autotune(nursd_batch* bt, const float* const* hist, float* const* I, void* ws, size_t ws_bytes,
                         void* stream) {
    NURSD_GUARD(nursd_batch_autotune_body(bt, hist, I, ws, ws_bytes, stream));
}

int nursd_batch_forward(nursd_batch* bt, const float* const* hist, float* const* I, void* ws, size_t ws_bytes,
                        void* stream) {
    NURSD_GUARD(nursd_batch_forward_body(bt, hist, I, ws, ws_bytes, stream));
}

int nursd_batch_tuning(const nursd_batch* bt, char* buf, size_t len) {
    NURSD_GUARD(nursd_batch_tuning_body(bt, buf, len));
}

}  // extern "C"
