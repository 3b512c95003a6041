/*
 * nursd.h -- C ABI of the MI355X NURSD / SRSD reconstruction library.
 *
 * Non-line-of-sight reconstruction by phasor-field Rayleigh-Sommerfeld
 * diffraction (RSD) with non-uniform relay sampling (NURSD) and the scaled
 * RSD (SRSD), after Sultan et al., "Optimized Sampling for Non-Line-of-Sight
 * Imaging Using Modified Fast Fourier Transforms":
 *   - measurement H(x_p, x_c, t) and relay positions in, as in the problem
 *     statement of the standard RSD section (phasor-field response,
 *     eq. PF_Response; RSD reconstruction, eq. PF_RSD_Defn);
 *   - wavelet parameters lambda_c and sigma of the Gaussian band-pass
 *     (eq. PFPacket_Omega_Supp);
 *   - output on a uniform voxel grid (eq. NURSD1), on per-plane voxel lists
 *     (eq. NURSD2 / eq. NURSD3) or on the scaled frustum (eq. SRSD_conv with
 *     the scaled FFT of eq. SFFT).
 *
 * Conventions
 *   Units: metres, seconds.  The relay plane is z = 0; planes have z > 0.
 *   Complex arrays are interleaved float pairs (re, im) = complex64.
 *   Every pointer named *_dev is device memory (HIP), owned by the caller;
 *   host arrays (z lists, bins, CSR offsets) are copied at plan creation.
 *   `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue work
 *   on that stream and do not synchronise it, except plan creation and
 *   nursd_plan_set_points, which read the relay positions back to the host.
 *   Errors: every int-returning call returns NURSD_OK (0) or a negative
 *   NURSD_ERR_* code; nursd_last_error() gives a message (thread-local).  No
 *   C++ exception crosses this interface.  A call that fails argument checks
 *   enqueues no work.
 *   Workspace: the caller allocates nursd_workspace_size() bytes of device
 *   memory (256-byte aligned) and passes it to the compute calls; its
 *   contents need not be preserved between calls.  The plan owns only small
 *   device tables (twiddles, deconvolution factors, binned relay lists).
 */
#ifndef NURSD_H
#define NURSD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NURSD_OK 0
#define NURSD_ERR_ARG (-1)              /* invalid argument or NULL pointer        */
#define NURSD_ERR_GEOMETRY (-2)         /* z <= 0, points outside the period, ...   */
#define NURSD_ERR_UNSUPPORTED_SIZE (-3) /* transform or time-axis size unsupported */
#define NURSD_ERR_WORKSPACE (-4)        /* workspace missing or misaligned          */
#define NURSD_ERR_HIP (-5)              /* a HIP runtime call failed                */
#define NURSD_ERR_UNIMPLEMENTED (-6)

#define NURSD_MODE_GRID 0   /* uniform voxel grid, NURSD-1                  */
#define NURSD_MODE_POINTS 1 /* per-plane voxel lists, NURSD-3 (or NURSD-2)  */
#define NURSD_MODE_SRSD 2   /* scaled RSD frustum                           */
#define NURSD_MODE_SRSD_POINTS 3 /* scaled RSD at per-plane voxel lists
                                    (eq. NURSD2_SRSD)                       */
#define NURSD_MODE_GRID3D 4 /* non-planar relays, 3D NURSD (eq. 3D_NURSD)  */

/* Phasor-field wavelet and temporal sampling (eq. PF_Response,
 * eq. PFPacket_Omega_Supp).  The F frequencies are DFT bins b of the T-bin
 * histograms, f_b = b / (T dt); by default F consecutive bins centred on
 * round(f_c T dt), f_c = c / lambda_c.  Each bin must satisfy 0 < b < T/2.
 * Weight of bin b: exp(-(f_b - f_c)^2 / (2 (sigma_rel f_c)^2)) e^{-j 2 pi f_b t0}. */
typedef struct {
    double lambda_c;      /* central wavelength [m]                              */
    double sigma_rel;     /* sigma_f / f_c; 0.2 is the paper's sigma = c/(5 lambda_c) */
    int32_t n_freq;       /* F >= 1                                              */
    int32_t n_time;       /* T, a power of two in [256, 8192] for nursd_phasor   */
    double dt;            /* bin width [s]                                       */
    double t0;            /* time of bin 0 [s]                                   */
    const int32_t* bins;  /* host array of F bins, or NULL for the centred band  */
    int32_t coherent;     /* 1: V = sum_b (...), I = |V|;  0: I = sum_b |F_b|     */
    int32_t kernel_inv_r; /* 1: plane-to-plane kernel G = e^{+jkr} / r, as printed
                             after eq. RSD_conv (nursd_default_options sets 1);
                             0: G = e^{+jkr}, the unit-amplitude phase of
                             eq. PF_RSD_Defn.  The illumination term has unit
                             amplitude either way.                              */
} nursd_wavelet;

/* Output sampling.
 * GRID:   voxel (ix, iy) of plane iz at (x0 + ix dx, y0 + iy dy, z[iz]);
 *         output arrays are [nz][ny][nx] (x fastest).
 * POINTS: plane iz owns voxels plane_ptr[iz] .. plane_ptr[iz+1]-1 of
 *         voxel_xy_dev ([V][2] float, device); dx, dy give the FFT pitch;
 *         outputs are [V].
 * SRSD:   uniform relay grid of nx x ny samples at pitch (dx, dy) around
 *         (x0, y0) (the GRID convention); plane iz is sampled at pitch
 *         (dx, dy) / alpha_iz, alpha_iz = alpha[iz] if alpha != NULL else
 *         zref / z[iz]; voxel (ix, iy) of plane iz lies at
 *         c + ((ix - nx/2) dx, (iy - ny/2) dy) / alpha_iz with
 *         c = (x0 + (nx/2) dx, y0 + (ny/2) dy).  Requires 0 < alpha <= 1,
 *         nx == ny, M >= 512 and M >= 2 (nx - 1) (the scaled DFT runs as
 *         two length-M convolutions per line; pad 2 always satisfies it);
 *         otherwise plan creation fails with UNSUPPORTED_SIZE.
 * SRSD_POINTS: the SRSD relay grid and scales, evaluated at per-plane voxel
 *         lists (plane_ptr, voxel_xy_dev as in POINTS) by a type-2 NUFFT in
 *         each plane's scaled frame (period M dx / alpha_iz around c), the
 *         fusion of the scaled RSD with NURSD-2 (eq. NURSD2_SRSD); outputs
 *         are [V].  Requires nx == ny and a transform size M >= 512.
 * GRID3D: the GRID voxel grid reconstructed from relay samples at depths
 *         z_l (relay_z_dev) on a non-planar surface (eq. 3D_NURSD): stage 1
 *         takes them to the plane z_mid by a 3D type-1 NUFFT onto
 *         M x M x mz3 modes (depth frame centred on z_mid, pitch dz3), times
 *         the 3D DFT of the 3D-RSD kernel e^{+jkr} (eq. 3d_rsd), read at
 *         z_mid; stage 2 propagates from z_mid to each voxel plane (depths
 *         z[iz] > z_mid) as GRID does.  mz3 = 0 picks the smallest power of
 *         two >= 8 with every |z_l - z_mid| <= mz3 dz3 / 4 (at most 64). */
typedef struct {
    int32_t mode;
    double x0, y0;
    double dx, dy;
    int32_t nx, ny;
    int32_t nz;
    const double* z;            /* host [nz], each > 0                          */
    const int32_t* plane_ptr;   /* host [nz+1] (POINTS, SRSD_POINTS)            */
    const float* voxel_xy_dev;  /* device [V][2] (POINTS, SRSD_POINTS)          */
    double zref;                /* SRSD, SRSD_POINTS                            */
    const double* alpha;        /* host [nz] (SRSD, SRSD_POINTS) or NULL        */
    double xp[3];               /* illumination point x_p                       */
    /* GRID3D: relay depths, the intermediate plane and the depth sampling */
    const float* relay_z_dev;   /* device [L] relay depths z_l                  */
    double z_mid;               /* intermediate plane z0 (< every voxel depth)  */
    double dz3;                 /* depth pitch of the 3D grid, 0 = dx           */
    int32_t mz3;                /* depth size of the 3D grid, 0 = auto          */
} nursd_geometry;

/* Numerical options. */
typedef struct {
    int32_t n_relay;     /* L >= 1                                              */
    double pad;          /* zero-padding factor, >= 1 (default 2)               */
    double sigma_os;     /* NUFFT oversampling; only 2.0 is supported           */
    double tol;          /* NUFFT tolerance (sets the spreading width), 1e-6    */
    int32_t M;           /* transform size, 0 = smallest that fits              */
    int32_t freq_chunk;  /* frequencies per propagation chunk, 0 = auto         */
    int32_t plane_chunk; /* planes per propagation chunk, 0 = auto              */
    /* Internal grid pitch dx / q (q >= 1; 0 or 1 = the voxel pitch).  The
     * standard RSD section samples the kernel at the relay rate; q > 1
     * samples the relay frame and the kernel q times finer than the voxels
     * (GRID, GRID3D: M >= pad * q * max(nx, ny); voxel (ix, iy) is grid point
     * (ix q - (nx q)/2, iy q - (ny q)/2) around the frame centre
     * c = (x0 + ((nx q)/2) dx / q, y0 + ((ny q)/2) dy / q); POINTS: FFT pitch
     * dx / q).  SRSD modes need q = 1 (else UNSUPPORTED_SIZE).               */
    int32_t upsample_q;
    /* Optional per-sample weights w_l (device [L] float, e.g. quadrature or
     * Voronoi areas; NULL = 1): every computation uses w_l P_l in place of
     * P_l (eq. NURSD1 applies the type-1 sum to the weighted samples).  The
     * weights are copied at plan creation; gradients (nursd_adjoint) are
     * taken with respect to the unweighted P and positions. */
    const float* weights_dev;
    /* Spreading tile of the type-1 NUFFT (NUFFT section, the blur step):
     * band rows x 100 + frequencies per workgroup, one of 108, 116, 208, 404,
     * 802, 1601 (108 = one fine row of 8 frequencies); 0 = the library's
     * choice.  Any tile gives bit-identical results (each fine-grid cell
     * takes its samples in the same order); a tile whose LDS footprint does
     * not fit the plan's fine grid is rejected with NURSD_ERR_ARG. */
    int32_t spread_tile;
} nursd_options;

typedef struct nursd_plan nursd_plan;
typedef struct nursd_batch nursd_batch;

/* Read-only facts about a plan (the periodic frame the operator is defined
 * on: relay x maps to 2 pi (x - cx) / (M dx)). */
typedef struct {
    int32_t M;            /* transform size                                    */
    int32_t Mf;           /* oversampled NUFFT grid size                       */
    int32_t n_freq;
    int32_t n_relay;
    int32_t kernel_width; /* ES spreading width                                */
    int32_t n_voxels;     /* voxels per output volume                          */
    double dx, dy;        /* grid pitch of the frame                           */
    double cx, cy;        /* frame centre                                      */
    double beta;          /* ES shape parameter                                */
    size_t workspace_bytes;
    int32_t freq_chunk;   /* frequencies per propagation launch               */
    int32_t plane_chunk;  /* depth planes per propagation launch              */
    int32_t depth3d;      /* depth size of the GRID3D stage-1 grid (else 0)   */
    int32_t upsample_q;   /* internal grid pitch = voxel pitch / upsample_q   */
} nursd_plan_info_t;

/* Fill the structs with defaults (pad 2, sigma_os 2, tol 1e-6, coherent,
 * kernel 1/r, sigma_rel 0.2, upsample_q 1, no weights).  Never fails for
 * non-NULL arguments. */
void nursd_default_options(nursd_wavelet* wl, nursd_geometry* geo, nursd_options* opt);

/* Create a plan: validates the geometry, chooses the periodic frame, bins
 * the relay samples for spreading and builds the device tables.
 * The frame follows the standard RSD section (the FFT convolution is
 * circular and needs zero padding, eq. Discrete_RSD_Conv) and the NUFFT
 * rescaling of the Non-Uniform RSD section (x~ = 2 pi (x - c) / (M dx) in
 * [-pi, pi)): M is the smallest supported size >= pad * q * max(nx, ny) with
 * every relay and voxel inside the period and every relay-voxel offset
 * strictly inside half a period.  The frequency bins follow the Gaussian
 * band of eq. PFPacket_Omega_Supp.  relay_xy_dev: device [L][2] float
 * (metres).  Synchronises `stream` once to read the positions (and weights).
 * Errors: ARG, GEOMETRY, UNSUPPORTED_SIZE, HIP. */
int nursd_plan_create(const nursd_wavelet* wl, const nursd_geometry* geo,
                      const nursd_options* opt, const float* relay_xy_dev,
                      void* stream, nursd_plan** out);

/* Replace the relay positions (same L); re-bins them.  Fails with GEOMETRY
 * (and keeps the previous positions) if a point leaves the plan's period or
 * a relay-voxel offset reaches half a period, the frame rule of plan
 * creation.  Synchronises `stream`. */
int nursd_plan_set_points(nursd_plan* plan, const float* relay_xy_dev, void* stream);

/* Facts of the frame and chunking chosen by nursd_plan_create. */
int nursd_plan_info(const nursd_plan* plan, nursd_plan_info_t* info);
/* Device workspace the compute calls of this plan need (bytes, to be
 * 256-byte aligned); the caller allocates and owns it. */
int nursd_workspace_size(const nursd_plan* plan, size_t* bytes);
void nursd_plan_destroy(nursd_plan* plan);

/* Step 1 alone: temporal phasor transform (eq. PF_Response with the
 * band-pass of eq. PFPacket_Omega_Supp).  hist_dev: [L][T] float, 8-byte
 * aligned (16-byte alignment with T = 2048 or 4096 takes the faster
 * one-wavefront-per-histogram kernel); P_dev: [F][L] complex64 output.
 * Errors: ARG (NULL or misaligned pointer), UNSUPPORTED_SIZE, HIP.  The same
 * alignment rule holds for every entry point that takes histograms. */
int nursd_phasor(nursd_plan* plan, const float* hist_dev, void* P_dev, void* stream);

/* Steps 2-3 alone: type-1 NUFFT of P_dev ([F][L] complex64) onto the
 * M x M modes (NUFFT section; spread, FFT, deconvolve).  U_dev: [F][M][M]
 * complex64, row index kx, column ky, both in FFT order (k mod M); the
 * stored value is U[k] / M^2.  Uses the workspace. */
int nursd_spectrum(nursd_plan* plan, const void* P_dev, void* U_dev, void* ws_dev,
                   size_t ws_bytes, void* stream);

/* Full reconstruction from histograms: steps 1-7.  Writes the complex volume
 * vol_dev (complex64, layout of the mode) and/or the intensity I_dev
 * (float, |V| for coherent plans, sum_b |F_b| otherwise); either may be NULL
 * but not both (vol_dev must be NULL for incoherent plans). */
int nursd_forward_hist(nursd_plan* plan, const float* hist_dev, void* vol_dev, float* I_dev,
                       void* ws_dev, size_t ws_bytes, void* stream);

/* nursd_forward_hist without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the workspace is a fixed device
 * array of NURSD_STATIC_SCRATCH_BYTES (512 MiB) inside the library, one per
 * GPU, held until the process ends; its address is looked up once per
 * device at plan creation.  The call allocates nothing and does not
 * synchronise.  Every call on one GPU shares that GPU's array and leaves its
 * contents behind (nothing in it needs to start at zero): calls that
 * overlap on one GPU (several streams or threads) race, so order them.
 * Errors: WORKSPACE when the plan's workspace exceeds the array (use
 * nursd_forward_hist), ARG while profiling is active (profiling creates
 * events), and those of nursd_forward_hist. */
#define NURSD_STATIC_SCRATCH_BYTES ((size_t)512 << 20)
int nursd_forward_hist_static(nursd_plan* plan, const float* hist_dev, void* vol_dev, float* I_dev, void* stream);

/* Reconstruction from phasors P_dev ([F][L] complex64): steps 2-7. */
int nursd_forward_phasor(nursd_plan* plan, const void* P_dev, void* vol_dev, float* I_dev,
                         void* ws_dev, size_t ws_bytes, void* stream);

/* Adjoint of the coherent map P -> V (GRID plans).  grad_vol_dev: [nz][ny][nx]
 * complex64, the upstream gradient dL/dRe V + j dL/dIm V.  Writes
 * grad_P_dev = A^H grad_vol ([F][L] complex64) and, if grad_xy_dev != NULL,
 * the relay-position gradient [L][2] float: Re sum_b conj(P_bl) d(...)/dx_l,
 * which needs P_dev.  The forward state is not stored: everything is
 * recomputed per frequency. */
int nursd_adjoint(nursd_plan* plan, const void* grad_vol_dev, const void* P_dev,
                  void* grad_P_dev, float* grad_xy_dev, void* ws_dev, size_t ws_bytes,
                  void* stream);

/* 4D light transport (eq. Video_Voxel_Freq_Offset): the coherent field of
 * every voxel at n_frames times t_j = t_first + j t_step [s],
 *   V(x_v, t_j) = sum_b e^{+j 2 pi f_b t_j} W_b(x_v),
 * where W_b is frequency b's field (back-propagation and illumination phase)
 * of a coherent GRID or SRSD plan; V(x_v, 0) is the forward volume.
 * Writes video_dev ([n_frames][nz][ny][nx] complex64) and/or video_I_dev
 * (same shape, |V|, float); either may be NULL but not both.  The plan is
 * processed in slabs of planes; each slab's per-frequency fields are kept in
 * the workspace, which must hold nursd_video_workspace_size bytes. */
int nursd_video_workspace_size(const nursd_plan* plan, size_t* bytes);
int nursd_forward_video(nursd_plan* plan, const void* P_dev, int32_t n_frames, double t_first, double t_step,
                        void* video_dev, float* video_I_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* Several illumination positions (the integral over x_p of eq. PF_RSD_Defn):
 * V = sum_k sum_b e^{+j k_b |x_v - x_p,k|} F_{k,b}(x_v), where F_{k,b} is the
 * back-propagation of the phasors measured under illumination k.  P_dev:
 * [K][F][L] complex64 (the plan's relay samples, one block per position);
 * xp_host: [K][3] positions, read before the call returns.  Each kernel
 * spectrum is generated once per (frequency, plane) and used for every
 * position.  Coherent GRID plans only; outputs as nursd_forward_phasor.
 * The workspace must hold nursd_multi_workspace_size bytes (the per-position
 * spectra are kept). */
int nursd_multi_workspace_size(const nursd_plan* plan, int32_t K, size_t* bytes);
int nursd_forward_multi(nursd_plan* plan, const void* P_dev, int32_t K, const double* xp_host, void* vol_dev,
                        float* I_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* Compression preprocessing (sampling-criteria section): phasors on a
 * uniform relay grid, in_dev [F][ny][nx] complex64, are kept on the lattice
 * of stride D along each axis and every grid point is filled from its nearest
 * kept sample (Euclidean distance; ties go to the lower index) -> out_dev,
 * same shape, a different buffer.  D = 1 copies.  Needs no plan. */
int nursd_subsample_nearest(const void* in_dev, void* out_dev, int32_t F, int32_t ny, int32_t nx, int32_t D,
                            void* stream);

/* Batched serving of many reconstructions of uneven size (not in the
 * paper: many phasor-field reconstructions, each eq. NURSD1 with the volume
 * of eq. PF_RSD_Defn, served together).  The plans may differ in relay
 * count, grid, frequency count, wavelength and transform size; all n plans
 * must be coherent GRID plans with T a power of two and evenly spaced
 * frequency bins.  Their reconstructions run as one HIP graph of grouped
 * persistent kernels: each grouped launch serves every plan of one kernel
 * type and size class, pulling work items from a device queue.  The
 * temporal transform, spreading and fine-grid passes of all plans are
 * grouped launches; plans with a transform size below a threshold are also
 * propagated by grouped launches, in R rounds each covering about 1/R of
 * every such plan's planes, while larger plans are propagated chunk by
 * chunk with ordinary launches inside the graph.  Grouped launches run in
 * one of three schedules: persistent workgroups fed by a device work queue,
 * persistent workgroups with a static stride, or one workgroup per work
 * block.  Plans whose kernels agree (transform size, grid pitch, 1/r form)
 * form a kernel class: the kernel spectrum quadrant of each distinct
 * (frequency, depth) pair of a class is generated once per batched forward
 * into a table in the workspace and read by the column passes of every
 * member plan (when the members use each pair at least 1.5 times on average
 * and the tables fit 24 GiB), instead of once per plan.  The plans must
 * outlive the batch and keep their relay positions while it exists.
 *
 * nursd_batch_create validates the plans, picks the default configuration
 * (work queue, threshold 512, the fewest rounds whose propagation scratch
 * fits 24 GiB) and allocates the batch's small device tables (work-item
 * tables sized for every configuration it may use, one queue counter per
 * grouped launch) and a pinned staging buffer; it launches nothing.  The
 * plans must outlive the batch.
 * nursd_batch_workspace_size: device workspace (256-byte aligned, owned by
 * the caller) that nursd_batch_forward and nursd_batch_autotune need; it
 * holds every plan's intermediates at once and, for a batch created with
 * autotune = 1, covers every configuration the tuner may pick.
 * nursd_batch_autotune (autotune = 1 batches only): times every candidate
 * configuration (threshold 256 / 512 / none x schedule x the two fewest
 * rounds whose grouped scratch fits 32 GiB) on the given inputs and keeps
 * the fastest.  It synchronises `stream`, like plan creation.
 * nursd_batch_forward: hist_dev[i] = [L_i][T_i] histograms of plan i,
 * I_dev[i] = [nz][ny][nx] intensity of plan i (float).  It allocates
 * nothing and does not synchronise: when the histogram, output or
 * workspace pointers differ from the previous call's, it rebuilds the work
 * tables on the host, copies them to the batch's table buffer on `stream`
 * (waiting only until this batch's previous table copy has left the pinned
 * staging buffer) and captures a new graph; then it launches the graph on
 * `stream`.  Calls on one batch must be ordered (one stream, or ordered by
 * the caller), since they share its table buffer and queue counters. */
int nursd_batch_create(nursd_plan* const* plans, int32_t n, int32_t autotune, void* stream,
                       nursd_batch** out);
int nursd_batch_workspace_size(const nursd_batch* batch, size_t* bytes);
int nursd_batch_autotune(nursd_batch* batch, const float* const* hist_dev, float* const* I_dev, void* ws_dev,
                         size_t ws_bytes, void* stream);
int nursd_batch_forward(nursd_batch* batch, const float* const* hist_dev, float* const* I_dev, void* ws_dev,
                        size_t ws_bytes, void* stream);
/* Configuration in use (R + 1000 * schedule + 10000 * threshold code +
 * 100000 * shared kernel tables; schedule 0 = work queue, 1 = static
 * stride, 2 = one workgroup per block; threshold code 0 = none chunk by
 * chunk, 1 = M >= 256, 2 = M >= 512),
 * number of launch records in the graph, the autotuner's candidates (same
 * encoding) and their times (ms per batch), workspace bytes.  Arrays may be
 * NULL; tried / tried_ms need room for 16 entries. */
int nursd_batch_info(const nursd_batch* batch, int32_t* budget, int32_t* launches, int32_t* n_tried,
                     int32_t* tried, float* tried_ms, size_t* workspace_bytes);
/* What the autotuner's second stage picked: after choosing the
 * configuration, nursd_batch_autotune tries the schedule variants of every
 * grouped launch class (kernel type and size) in turn -- the spreading tile
 * (fine rows per band 4 / 8 / 16 and frequencies per workgroup 1 / 2 / 4,
 * within LDS), lines per workgroup of the fine-grid y transform (2 / 4 / 8)
 * and waves per block of the kernel-row, column and last passes (4 / 8,
 * 2 / 4 / 8, 4 / 8) -- timing that class's launches with events in an
 * eager run, and keeps the fastest; picks are cached per process by (kind,
 * size, log2 of the launch's work).  Writes one line per class
 * ("kind/size: choice (best ms, default ms)", "; "-separated, truncated to
 * len) into buf. */
int nursd_batch_tuning(const nursd_batch* batch, char* buf, size_t len);
void nursd_batch_destroy(nursd_batch* batch);

/* Per-kernel timing with HIP events, for profiling and roofline reports.
 * nursd_profile_begin starts recording an event pair around every launch
 * of the stages selected by stage_mask (bit i = stage i, NURSD_STAGE_*);
 * nursd_profile_end waits for the recorded events, writes the summed
 * milliseconds and the launch count per stage (arrays of NURSD_NUM_STAGES)
 * and stops recording.  Events are recorded on the stream of each call. */
#define NURSD_STAGE_PHASOR 0
#define NURSD_STAGE_SPREAD 1
#define NURSD_STAGE_FINE_Y 2
#define NURSD_STAGE_KERNEL_ROWS 3
#define NURSD_STAGE_PROPAGATE_COLS 4
#define NURSD_STAGE_PROPAGATE_ROWS 5
#define NURSD_STAGE_CHIRP_ROWS 6
#define NURSD_STAGE_RELAY_GRID 7
#define NURSD_STAGE_TYPE2 8
#define NURSD_STAGE_ADJOINT 9
#define NURSD_STAGE_VIDEO 10
#define NURSD_STAGE_NURSD3D 11
#define NURSD_NUM_STAGES 16
int nursd_profile_begin(nursd_plan* plan, uint32_t stage_mask);
int nursd_profile_end(nursd_plan* plan, double* ms, int32_t* calls);

const char* nursd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NURSD_H */
