// Kernel parameter blocks and launcher declarations shared by the HIP
// translation units and the host-side C-ABI implementation.
#pragma once
#include <hip/hip_runtime.h>
#include "host_plan.hpp"
#include "persistent.hpp"
#include <cstddef>
#include <cstdint>

namespace nursd {

constexpr double kC = 299792458.0;   // speed of light [m/s]
constexpr int kMaxLog = 13;          // twiddle tables for N = 2^0 .. 2^12

// Fine-grid rows per spreading band (one band of one frequency fills LDS).
constexpr int spread_band_rows(int) { return 8; }
// Frequencies spread by one workgroup: the kernel weights of a sample are
// computed once and applied to each of them (one LDS tile per frequency).
constexpr int spread_freqs(int Mf) { return Mf <= 1024 ? 2 : 1; }
struct TwTables {
    const float2* t[kMaxLog];   // t[n][m] = e^{-2 pi j m / 2^n}
};

// ---------------------------------------------------------------- step 1
struct PhasorArgs {
    const float* hist;     // [L][T]
    float2* P;             // [F][L]
    int L, T, F;
    const int* bins;       // [F]
    const float2* wt;      // [F] Gaussian weight * e^{-j 2 pi f t0}
    const float2* tb;      // [F] e^{-j 2 pi b / T}
    const float2* tw;      // twiddles of size T/2
};
hipError_t launch_phasor(const PhasorArgs& a, hipStream_t s);

// ---------------------------------------------------------------- steps 2-3
struct SpreadArgs {
    int var = 0;                  // spreading tile (spread_var); the lists are binned for its rows
    const float2* P;              // [F][L] (frequency-major)
    const float* wts;             // [L] per-sample weights multiplying P, or NULL
    const SpreadEntry* ent;       // entries sorted by band, then u
    const int* band_ptr;          // [nbands + 1]
    const int* wave_rng;          // [nbands][kSpreadWaves][4]: entry range, then column range, of each wave
    float2* T1;                   // [Fc][Mf/BR][M][BR]: x-transformed bands of BR fine rows,
                                  // each band's M kept modes with its rows innermost
    const float* decx;            // [M] (-1)^kx / (phihat(kx) M^2), FFT order
    const float2* tw;             // twiddles of size Mf
    int M, Mf, L, w;
    float beta, half_w;
    int b0, nb;                   // frequency range of this launch
};
hipError_t launch_spread_xfft(const SpreadArgs& a, hipStream_t s);

struct FineYArgs {
    const float2* T1;             // [Fc][Mf/br][M][br], as the spreading wrote it
    float2* U;                    // [F][M][M] (kx row, ky column, FFT order)
    const float* decy;            // [M]
    const float2* tw;             // size Mf
    int M, Mf;
    int b0, nb;
    int br;                       // band rows of the spreading tile that wrote T1
};
hipError_t launch_fine_y(const FineYArgs& a, hipStream_t s);

// ---------------------------------------------------------------- step 4-7
// Planes of a chunk: plane p -> frequency b = b0 + p / nz_c, depth iz = z0 + p % nz_c.
struct ChunkGeom {
    int b0, nb;         // frequency range
    int z0, nzc;        // plane range
    const double* f;    // [F] frequencies [Hz]
    const double* z;    // [Z] depths [m]
    const double* pitch_x;  // per-plane kernel pitch (SRSD) or NULL (use dx)
    const double* pitch_y;
    double dx, dy;      // kernel sampling pitch
    int uni;            // 1: f[b0 + i] = f[b0] + i * df for the whole chunk
    double df;          // frequency step of the chunk when uni = 1
};

struct P1Args {
    ChunkGeom g;
    float2* Bt;         // [planes][M/2+1][BS]
    int M, BS;
    const float2* tw;   // size M
    int plain = 0;      // 1: the 3D-RSD kernel e^{+jkr} (no 1/r; r = 0 allowed)
};
hipError_t launch_kernel_rows(const P1Args& a, hipStream_t s);

struct P2Args {
    ChunkGeom g;
    const float2* Bt;   // [planes][M/2+1][BS]
    const float2* U;    // [F][M][M]
    float2* Yt;         // [planes][M][ny]: kx line s, then window row iy
    int M, BS, ny;
    const float2* tw;
    int q = 1;          // window row iy is grid row iy q - (ny q)/2 (upsampled frame)
    // Batched mode: the kernel quadrant of frequency b and plane iz is plane
    // kidx[b * kz + iz] of Bt, a table shared by the scenes of one transform
    // size and pitch; NULL: plane p of the chunk.
    const int* kidx = nullptr;
    int kz = 0;
};
hipError_t launch_propagate_cols(const P2Args& a, hipStream_t s);

// Batched mode: the column pass of one kernel table plane for several
// scenes.  Item i (grid y) transforms the kernel lines of table plane kp[i]
// once and, for each user u in [user_ptr[i], user_ptr[i + 1]), multiplies
// them by the user's spectrum rows U[+-kx] and writes the inverse transform
// of the window rows to the user's output plane Yt ([M][ny], as P2Args).
struct P2MUser {
    const float2* U;    // [M][M] spectrum of the user's frequency
    float2* Yt;         // [M][ny] output plane
    int ny, q;
};
struct P2MArgs {
    const float2* Bt;       // kernel table [planes][M/2+1][BS]
    const int* kp;          // [items] table plane of each item
    const int* user_ptr;    // [items + 1]
    const P2MUser* users;
    // Work blocks (item, kx block) by block index.  The dispatcher deals
    // block indices to the 8 XCDs in turn, so the host interleaves eight kx
    // blocks of one frequency at a time: each XCD then walks the depths of
    // one (frequency, kx block) back to back and reads the users' spectrum
    // rows from its L2, while the XCDs stay balanced block by block.
    const int2* blk;
    int M, BS;
    const float2* tw;
};
// halfy: every user's window satisfies ny q <= M/2 (rows |m| >= M/4 unused).
hipError_t launch_propagate_cols_multi(const P2MArgs& a, int nblk, bool halfy, hipStream_t s);
int grid_x_propagate_cols_multi(int M);

struct P3Args {
    ChunkGeom g;
    const float2* Yt;   // [planes][M][ny]: kx line s, then window row iy
    float2* V;          // [Z][ny][nx] (may be NULL for incoherent)
    float* I;           // [Z][ny][nx] or NULL
    int M, nx, ny;
    double xc, yc;      // voxel (ix, iy) at (xc + (ix q - (nx q)/2) px, yc + (iy q - (ny q)/2) py)
    double xp0, xp1, xp2;
    int first, last, coherent;
    const float2* tw;
    // Per-frequency field output (4D video): when set, each frequency's
    // phased contribution is stored at field[b][iz - field_z0][iy][ix]
    // (frequency stride field_nz * ny * nx) instead of being summed.
    float2* field;
    int field_z0, field_nz;
    int q = 1;          // grid points per voxel pitch (upsampled frame)
};
hipError_t launch_propagate_rows(const P3Args& a, hipStream_t s);

// ---------------------------------------------------------------- 4D video
// V(x, t_j) = sum_b e^{+j 2 pi f_b t_j} W_b(x) for the planes of one slab,
// t_j = t_first + j t_step (eq. Video_Voxel_Freq_Offset).
struct VideoArgs {
    const float2* field;     // [F][field_nz][nvp] per-frequency fields of the slab
    const double* f;         // [F] frequencies [Hz]
    float2* V;               // [T][nz][nvp] complex video or NULL
    float* I;                // [T][nz][nvp] |V| or NULL
    int F, field_nz, nzc, z0, nz, nvp, T;
    double t_first, t_step;
};
hipError_t launch_video(const VideoArgs& a, hipStream_t s);

// ---------------------------------------------------------------- 3D NURSD
// Stage 1 (eq. 3D_NURSD): with W_p(l) the depth weights of relay l for depth
// index p of the 3D grid, the spectrum at the intermediate plane is
//   U0[k] = sum_p Ghat(p dz)[k] NUFFT2{P_l W_p(l)}[k].
struct ModulateArgs {
    const float2* P;      // [F][L] phasors
    const float2* W;      // [Mz][L] depth weights
    float2* Q;            // [Mz][nb][L] modulated phasors
    int L, Mz, b0, nb;
};
hipError_t launch_modulate(const ModulateArgs& a, hipStream_t s);

struct Stage1Args {
    ChunkGeom g;          // frequencies b0 .. b0+nb-1, planes = the Mz depths
    const float2* Bt;     // [nb * Mz][M/2+1][BS] kernel quadrant rows (plain kernel)
    const float2* Ut;     // [Mz][nb][M][M] spectra of the modulated phasors (/ M^2, FFT order)
    float2* U0;           // [F][M][M] stage-1 spectra (/ M^2, FFT order)
    int M, BS, Mz;
    const float2* tw;
};
hipError_t launch_stage1_reduce(const Stage1Args& a, hipStream_t s);

// ---------------------------------------------------------------- compression
hipError_t launch_subsample_nearest(const float2* in, float2* out, int F, int ny, int nx, int D, hipStream_t s);

// ---------------------------------------------------------------- step 6
struct RelayGridArgs {
    const float2* U;        // [F][M][M] spectra (scaled by M^-2)
    float2* Tg;             // [nb][M][N] scratch
    float2* u;              // [F][N][N] uniform relay grid
    int M, N;
    int b0, nb;
    const float2* tw_m;
};
hipError_t launch_relay_grid(const RelayGridArgs& a, hipStream_t s);

struct ChirpArgs {
    ChunkGeom g;
    const float2* u;        // [F][N][N]
    float2* S1t;            // [planes][M][N] row-scaled spectra, transposed
    const float2* Bt;       // [planes][M/2+1][BS] kernel quadrant rows (pitch d/alpha)
    float2* Yt;             // [planes][M][ny]
    int M, N, BS, ny;
    const double* alpha;    // [Z]
    const float2* hhat;     // [Z][2][M] chirp spectra of the two output halves / (M * M)
    const float2* chirp;    // [Z][M] e^{-j pi alpha m^2 / M}, m = j - M/2
    const float2* tw_m;     // twiddles of size M
    const float2* tw_lb;    // twiddles of size 2M (oversampled type-2 line)
    float2* T2;             // [planes][M][2M] (voxel-list output only)
    const float* dec;       // [M] (-1)^k / phihat(k), FFT order (voxel-list output only)
    const int* row_lo;      // [Z] reachable fine rows of each plane (voxel-list output only)
    const int* row_hi;
};
hipError_t launch_chirp_rows(const ChirpArgs& a, hipStream_t s);
hipError_t launch_chirp_cols(const ChirpArgs& a, hipStream_t s);
// Scaled spectrum times kernel spectrum, deconvolved and zero-padded to the
// oversampled line, inverse FFT along y -> T2 (type-2 output of eq. NURSD2_SRSD).
hipError_t launch_chirp_type2_cols(const ChirpArgs& a, hipStream_t s);

// xcd_contiguous (persistent.hpp) maps workgroup ids to XCD-contiguous runs of work items.

// Load of data read for the last time (an intermediate the next kernels do
// not need): marked non-temporal, so the caches evict it first and keep what
// the next kernel reads.
__device__ __forceinline__ float2 load_last(const float2* p) {
    typedef float v2f __attribute__((ext_vector_type(2)));
    const v2f t = __builtin_nontemporal_load(reinterpret_cast<const v2f*>(p));
    return make_float2(t.x, t.y);
}

// ---------------------------------------------------------------- step 5 (voxel lists)
// Fine rows the type-2 row pass transforms per block; the column passes store
// T2 only in the bands of kType2RowBand rows from a plane's first reachable row.
constexpr int kType2RowBand = 8;
__device__ __forceinline__ bool type2_row_stored(int jy, int lo, int hi, int mf) {
    const int nrows = ((hi - lo) / kType2RowBand + 1) * kType2RowBand;
    return ((jy - lo) & (mf - 1)) < nrows;
}
struct Type2Args {
    ChunkGeom g;
    const float2* Bt;        // [planes][M/2+1][BS]
    const float2* U;         // [F][M][M]
    float2* T2;              // [planes][M][Mf]
    float2* V;               // [V] or NULL
    float* I;                // [V] or NULL
    const float* dec;        // [M] (-1)^k / phihat(k), FFT order
    const float2* tw_m;
    const float2* tw_f;
    int M, Mf, BS, w;
    float beta;
    double cx, cy;
    double xp0, xp1, xp2;
    const int* plane_ptr;    // [Z+1]
    const float* voxel_xy;   // [V][2]
    const int* row_lo;       // [Z] first fine row any voxel of the plane reaches (may be < 0)
    const int* row_hi;       // [Z] last such row
    // interpolation entries: one per (voxel, band of kType2RowBand fine rows
    // from row_lo its taps reach), sorted by plane, then band, then voxel
    const int* plane_band;   // [Z+1] first band of each plane in band_ptr
    const int* band_ptr;     // [bands + 1] entry range of each band
    const int* ent_vox;      // [n_lent] voxel of each entry
    const int* vox_ent;      // [V][2] entries of each voxel (the second -1 if one)
    float2* part;            // [frequencies of the chunk][n_lent] partial sums
    int n_lent;
    int max_vox;             // largest voxel count of a plane
    int first, last, coherent;
};
hipError_t launch_type2(const Type2Args& a, hipStream_t s);
// The fine-grid and interpolation steps alone (T2 already filled).
hipError_t launch_type2_fine(const Type2Args& a, hipStream_t s);

// ---------------------------------------------------------------- step 8
struct AdjArgs {
    ChunkGeom g;
    const float2* gV;        // [Z][ny][nx] upstream gradient
    float2* Rt;              // [planes][M][ny]
    const float2* Bt;        // [planes][M/2+1][BS]
    float2* St;              // [F][M][M] adjoint spectra (FFT order)
    float2* T3;              // [nb][3][M][Mf]
    float2* G3;              // [nb][3][Mf][Mf]
    const float2* P;         // [F][L] (for the position gradient)
    float2* grad_P;          // [F][L]
    float* grad_xy;          // [L][2] or NULL
    const float* relay;      // [L][2]
    const float2* tw_m;
    const float2* tw_f;
    const float* dec;        // [M] (-1)^k / phihat(k)
    int M, Mf, BS, nx, ny, L, w;
    float beta;
    float kscale_x, kscale_y;    // 2 pi / (M dx), 2 pi / (M dy)
    double xc, yc;           // grid point with index 0 (voxel window centre)
    double cx, cy;           // frame centre (relay rescaling)
    double xp0, xp1, xp2;
    int relay_row_lo, relay_row_hi;
    int first;               // first plane chunk: St is written, else accumulated
    int first_b;             // first frequency chunk: grad_xy is written, else accumulated
    int q = 1;               // window index i is grid index i q - (n q)/2
    const float* wts = nullptr;  // [L] per-sample weights of the forward, or NULL
};
hipError_t launch_adjoint_planes(const AdjArgs& a, hipStream_t s);
hipError_t launch_adjoint_type2(const AdjArgs& a, hipStream_t s);

// ---------------------------------------------------------------- grouped launches
hipError_t launch_phasor_grouped(int T, int F_max, const Group<PhasorArgs>& g, hipStream_t s);
// Grouped launches of the batched mode.  Each takes a schedule variant of its
// kernel, which the batch's tuner picks per size class:
//   spreading: spread_var(BR, NF) = BR * 100 + NF (band rows, frequencies
//     per workgroup; 0 = spread_band_rows / spread_freqs), valid where
//     spread_var_ok (also the plans' own spreading tile);
//   fine y: lines per workgroup (2, 4, 8; 64 threads per line);
//   kernel rows: waves per block (4, 8); column pass: waves per block
//   (2, 4, 8); last pass: waves per block (4, 8).
constexpr int spread_var(int br, int nf) { return br * 100 + nf; }
constexpr int spread_var_rows(int var, int Mf) { return var ? var / 100 : spread_band_rows(Mf); }
constexpr int spread_var_freqs(int var, int Mf) { return var ? var % 100 : spread_freqs(Mf); }
bool spread_var_ok(int Mf, int var);
bool spread_var_plain_ok(int Mf, int var);   // variants of the plain (per-plan) launch
// The spreading and fine-y launches keep the modes of a sigma = 2 grid: every
// item has Mf = 2M, as every plan's fine grid does (launch_spread_xfft checks).
hipError_t launch_spread_xfft_grouped(int Mf, int var, const Group<SpreadArgs>& g, hipStream_t s);
hipError_t launch_fine_y_grouped(int Mf, int lines, const Group<FineYArgs>& g, hipStream_t s);
hipError_t launch_kernel_rows_grouped(int M, int nw, const Group<P1Args>& g, hipStream_t s);
hipError_t launch_propagate_cols_grouped(int M, bool halfy, int nw, const Group<P2Args>& g, hipStream_t s);
hipError_t launch_propagate_rows_grouped(int M, bool half, int nw, const Group<P3Args>& g, hipStream_t s);
int grid_x_kernel_rows(int M, int nw);
int grid_x_propagate_cols(int M, int nw);
int rows_per_block_propagate(int M, int nw);
int fine_y_lines();
int phasor_group();
hipError_t launch_zero_counters(int* c, int n, hipStream_t s);

}  // namespace nursd
