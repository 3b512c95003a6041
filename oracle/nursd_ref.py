"""FP64 CPU oracle for NURSD and SRSD.

TEST INFRASTRUCTURE ONLY.  This module is imported by tests/, by
__graft_entry__.smoke() and by bench.py's cpu_baseline leg, and by nothing
else.  The GPU product path never imports, links or calls it, and it shares
no code with the GPU path (no kernels, headers, tables or helpers).

Every fast transform of the method is replaced here by its direct
definition, evaluated in float64 / complex128:
  * the temporal phasor transform by a direct DFT over the time bins,
  * NUFFT type 1 / type 2 by the direct non-uniform sums (NUDFT-1 / NUDFT-2),
  * each spatial FFT by a direct separable DFT over the centred index set I_M,
  * the scaled FFT (chirp-z) by the direct scaled DFT.
There is no spreading kernel, no FFT and no chirp factorisation in this file.
A matrix product is used as a primitive to evaluate the separable sums.

Conventions (readings of the paper where its text is ambiguous or silent):
  * temporal transform e^{-j 2 pi f t}; back-propagation multiplies by
    e^{+j k r} for both the relay->voxel kernel and the illumination term,
    with k = 2 pi f / c;
  * RSD kernel G(p, z) = e^{+j k r} / r, r = sqrt(|p|^2 + z^2) (standard RSD
    section, kernel of the plane-to-plane convolution); inv_r=False drops the
    1/r, the unit-amplitude phase of eq. PF_RSD_Defn;
  * the frame is sampled at pitch (voxel pitch) / q, q = upsample_q >= 1
    (q = 1: the kernel sampled at the relay/voxel rate, standard RSD
    section); voxel i of a window of n is grid index i q - (n q)//2;
  * optional per-sample weights w_l multiply the phasors (no density
    compensation unless weights are given);
  * Gaussian band-pass weight exp(-(f - f_c)^2 / (2 sigma_f^2)),
    sigma_f = 0.2 f_c, on F consecutive DFT bins centred on round(f_c / df);
  * coherent sum over frequencies, intensity = |V|;
  * I_n = {-n/2, ..., n/2 - 1} (the paper's centred index set);
  * output of the scaled RSD at pitch dx / alpha(z), alpha(z) = z_ref / z.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

C_LIGHT = 299_792_458.0
SUPPORTED_M = (64, 128, 256, 512, 1024)


def centered(n: int) -> np.ndarray:
    """The centred index set I_n = {l in Z : -n/2 <= l < n/2} (2D DFT section)."""
    return np.arange(-(n // 2), (n + 1) // 2)


# ---------------------------------------------------------------------------
# Step 1: temporal phasor transform (phasor-field response, eq. PF_Response,
# with the Gaussian band-pass illumination of eq. PFPacket_Omega_Supp).
# ---------------------------------------------------------------------------
def wavelet_bins(lambda_c: float, n_time: int, dt: float, n_freq: int, bins=None):
    """DFT bins b and their frequencies f_b = b / (T dt).  Default: F consecutive
    bins centred on round(f_c / df), f_c = c / lambda_c.  Every bin must lie in
    (0, T/2)."""
    df = 1.0 / (n_time * dt)
    if bins is None:
        k0 = int(round((C_LIGHT / lambda_c) / df))
        bins = k0 - n_freq // 2 + np.arange(n_freq)
    bins = np.asarray(bins, dtype=np.int64)
    if np.any(bins <= 0) or np.any(2 * bins >= n_time):
        raise ValueError("frequency bin outside (0, T/2)")
    return bins, bins * df


def phasor_weights(f: np.ndarray, lambda_c: float, sigma_rel: float, t0: float) -> np.ndarray:
    """w(f) e^{-j 2 pi f t0}: the Gaussian illumination spectrum
    exp(-(f - f_c)^2 / (2 sigma_f^2)) with sigma_f = sigma_rel * f_c, times the
    phase that moves the time origin from bin 0 to t = 0."""
    fc = C_LIGHT / lambda_c
    sf = sigma_rel * fc
    return np.exp(-((f - fc) ** 2) / (2.0 * sf * sf)) * np.exp(-2j * np.pi * f * t0)


def temporal_phasor(hist: np.ndarray, bins: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """P[j][l] = weights[j] * sum_t H[l][t] e^{-j 2 pi b_j t / T}  (direct DFT).
    hist: [L][T] real; returns complex128 [F][L]."""
    h = np.asarray(hist, dtype=np.float64)
    T = h.shape[1]
    t = np.arange(T, dtype=np.float64)
    E = np.exp(-2j * np.pi * np.outer(t, np.asarray(bins, dtype=np.float64)) / T)  # [T][F]
    return (h @ E).T * np.asarray(weights)[:, None]


# ---------------------------------------------------------------------------
# Step 2: periodic frame.  The FFT-based propagation is a circular
# convolution over a period of M samples; with enough zero padding it equals
# the linear convolution of the RSD integral for on-grid data.
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Frame:
    M: int           # transform size per axis
    dx: float        # grid pitch along x [m]
    dy: float
    cx: float        # grid point with index 0 [m]
    cy: float
    q: int = 1       # grid points per voxel pitch (uniform-grid modes)

    @property
    def Lx(self) -> float:
        return self.M * self.dx

    @property
    def Ly(self) -> float:
        return self.M * self.dy


def _fits(M, dx, dy, cx, cy, relay_xy, vox_lo, vox_hi):
    """Relay points inside the period around (cx, cy), voxels inside it, and
    every relay-voxel difference inside (-L/2, L/2)."""
    r = np.asarray(relay_xy, dtype=np.float64)
    for axis, d, c in ((0, dx, cx), (1, dy, cy)):
        L = M * d
        rmin, rmax = r[:, axis].min(), r[:, axis].max()
        vmin, vmax = vox_lo[axis], vox_hi[axis]
        if rmin - c < -L / 2 or rmax - c >= L / 2:
            return False
        if vmin - c < -L / 2 or vmax - c >= L / 2:
            return False
        if max(vmax - rmin, rmax - vmin) >= L / 2:
            return False
    return True


def choose_frame(mode: str, relay_xy, *, x0=0.0, y0=0.0, dx=1.0, dy=1.0, nx=0, ny=0,
                 voxel_xy=None, pad: float = 2.0, sizes=SUPPORTED_M, q: int = 1) -> Frame:
    """Frame rule (zero padding of the standard RSD section):
      grid / srsd: pitch = voxel pitch / q, index 0 at grid point
                   x0 + ((nx q)//2) pitch (voxel (nx//2, ny//2) when q = 1), M the
                   smallest supported size >= pad * q * max(nx, ny) that passes _fits;
      points:      pitch = dx / q, index 0 at the centre of the joint bounding box
                   of relays and voxels, M the smallest supported size passing _fits."""
    if mode in ("grid", "srsd"):
        gx, gy = dx / q, dy / q
        cx = x0 + ((nx * q) // 2) * gx
        cy = y0 + ((ny * q) // 2) * gy
        lo = (x0, y0)
        hi = (x0 + (nx - 1) * dx, y0 + (ny - 1) * dy)
        mmin = pad * max(nx, ny) * q
    elif mode == "points":
        r = np.asarray(relay_xy, dtype=np.float64)
        v = np.asarray(voxel_xy, dtype=np.float64)
        lo = (v[:, 0].min(), v[:, 1].min())
        hi = (v[:, 0].max(), v[:, 1].max())
        cx = 0.5 * (min(lo[0], r[:, 0].min()) + max(hi[0], r[:, 0].max()))
        cy = 0.5 * (min(lo[1], r[:, 1].min()) + max(hi[1], r[:, 1].max()))
        gx, gy = dx / q, dy / q
        mmin = 0
    else:
        raise ValueError(mode)
    for M in sizes:
        if M >= mmin and _fits(M, gx, gy, cx, cy, relay_xy, lo, hi):
            return Frame(M, gx, gy, cx, cy, q)
    raise ValueError("no supported transform size fits the geometry")


def window_index(n: int, q: int = 1) -> np.ndarray:
    """Grid indices (around the frame centre) of the n voxels of a window:
    i q - (n q)//2 for i = 0 .. n-1 (every q-th grid point)."""
    return np.arange(n) * q - (n * q) // 2


def rescale(x: np.ndarray, c: float, period: float) -> np.ndarray:
    """Map positions to [-pi, pi): x~ = 2 pi (x - c) / period (NUFFT section)."""
    return 2.0 * np.pi * (np.asarray(x, dtype=np.float64) - c) / period


# ---------------------------------------------------------------------------
# Step 3: NUFFT type 1 / type 2 by their direct definitions (NUFFT section).
# ---------------------------------------------------------------------------
def nudft1(P: np.ndarray, xt: np.ndarray, yt: np.ndarray, M: int) -> np.ndarray:
    """U[kx][ky] = sum_l P[l] e^{-j (kx x~_l + ky y~_l)}, (kx, ky) in I_M^2.
    P: [L] or [F][L]; returns [M][M] or [F][M][M] (row = kx, column = ky)."""
    k = centered(M).astype(np.float64)
    Ex = np.exp(-1j * np.outer(k, xt))          # [M][L]
    Ey = np.exp(-1j * np.outer(k, yt))          # [M][L]
    P = np.asarray(P, dtype=np.complex128)
    if P.ndim == 1:
        return (Ex * P[None, :]) @ Ey.T
    return np.stack([(Ex * p[None, :]) @ Ey.T for p in P])


def nudft2(U: np.ndarray, xt: np.ndarray, yt: np.ndarray) -> np.ndarray:
    """u[l] = sum_{k in I_M^2} U[kx][ky] e^{+j (kx x~_l + ky y~_l)}."""
    M = U.shape[-1]
    k = centered(M).astype(np.float64)
    Ex = np.exp(1j * np.outer(xt, k))           # [L][M]
    Ey = np.exp(1j * np.outer(yt, k))           # [L][M]
    return np.einsum("lk,km,lm->l", Ex, U, Ey, optimize=True)


# ---------------------------------------------------------------------------
# Steps 4-5: RSD kernel spectrum and inverse transform (eq. RSD_conv,
# eq. Discrete_RSD_Conv and eq. NURSD1).
# ---------------------------------------------------------------------------
def kernel_samples(f: float, z: float, M: int, dx: float, dy: float, inv_r: bool = True) -> np.ndarray:
    """G(m dx, n dy, z) = e^{+j 2 pi f r / c} / r (or without the 1/r when
    inv_r is False) for (m, n) in I_M^2; [m][n]."""
    m = centered(M).astype(np.float64)
    X = (m * dx)[:, None]
    Y = (m * dy)[None, :]
    r = np.sqrt(X * X + Y * Y + z * z)
    g = np.exp(2j * np.pi * f * r / C_LIGHT)
    return g / r if inv_r else g


def dft_matrix(M: int, sign: float = -1.0, rows=None, cols=None) -> np.ndarray:
    """E[a][b] = exp(sign * 2 pi j * rows[a] * cols[b] / M)."""
    rows = centered(M) if rows is None else np.asarray(rows)
    cols = centered(M) if cols is None else np.asarray(cols)
    return np.exp(sign * 2j * np.pi * np.outer(rows, cols).astype(np.float64) / M)


def dft2(g: np.ndarray) -> np.ndarray:
    """Ĝ[kx][ky] = sum_{(m,n) in I_M^2} g[m][n] e^{-2 pi j (kx m + ky n) / M}."""
    D = dft_matrix(g.shape[0], -1.0)
    return D @ g @ D.T


def idft2_at(X: np.ndarray, mx: np.ndarray, my: np.ndarray) -> np.ndarray:
    """F[a][b] = M^{-2} sum_k X[kx][ky] e^{+2 pi j (kx mx[a] + ky my[b]) / M}."""
    M = X.shape[0]
    Ax = dft_matrix(M, +1.0, rows=mx)           # [len(mx)][M]
    Ay = dft_matrix(M, +1.0, rows=my)
    return (Ax @ X @ Ay.T) / (M * M)


def illumination_phase(f: float, x, y, z, xp) -> np.ndarray:
    """e^{+j 2 pi f |x_v - x_p| / c} (illumination leg of eq. PF_RSD_Defn)."""
    d = np.sqrt((x - xp[0]) ** 2 + (y - xp[1]) ** 2 + (z - xp[2]) ** 2)
    return np.exp(2j * np.pi * f * d / C_LIGHT)


def nursd_grid(P, relay_xy, f, frame: Frame, grid, xp, coherent=True, intensity=False, inv_r=True,
               weights=None):
    """NURSD-1 onto a uniform voxel grid (eq. NURSD1, volume formation of
    eq. PF_RSD_Defn).  P: [F][L]; weights: optional [L] factors w_l applied to
    every P[b][l]; the voxels are every q-th point of the frame
    (window_index).  Returns V complex [Z][ny][nx] (coherent) or sum_b |F_b|
    (incoherent)."""
    if weights is not None:
        P = np.asarray(P) * np.asarray(weights, dtype=np.float64)[None, :]
    xt = rescale(relay_xy[:, 0], frame.cx, frame.Lx)
    yt = rescale(relay_xy[:, 1], frame.cy, frame.Ly)
    mx = window_index(grid.nx, frame.q)
    my = window_index(grid.ny, frame.q)
    xs = frame.cx + mx * frame.dx
    ys = frame.cy + my * frame.dy
    z = np.asarray(grid.z, dtype=np.float64)
    out = np.zeros((len(z), grid.ny, grid.nx), dtype=np.float64 if not coherent else np.complex128)
    for b, fb in enumerate(f):
        U = nudft1(P[b], xt, yt, frame.M)
        for iz, zz in enumerate(z):
            Gh = dft2(kernel_samples(fb, zz, frame.M, frame.dx, frame.dy, inv_r))
            Fz = idft2_at(U * Gh, mx, my).T                    # [ny][nx]
            if coherent:
                ph = illumination_phase(fb, xs[None, :], ys[:, None], zz, xp)
                out[iz] += ph * Fz
            else:
                out[iz] += np.abs(Fz)
    return np.abs(out) if (coherent and intensity) else out


def nursd_points(P, relay_xy, f, frame: Frame, z, plane_ptr, voxel_xy, xp, inv_r=True):
    """NURSD-3: NUDFT-1 in, NUDFT-2 out at per-plane voxel lists (eq. NURSD3,
    which reduces to eq. NURSD2 for on-grid relays).  Returns V complex [V]."""
    xt = rescale(relay_xy[:, 0], frame.cx, frame.Lx)
    yt = rescale(relay_xy[:, 1], frame.cy, frame.Ly)
    vx = np.asarray(voxel_xy[:, 0], dtype=np.float64)
    vy = np.asarray(voxel_xy[:, 1], dtype=np.float64)
    out = np.zeros(len(vx), dtype=np.complex128)
    M = frame.M
    for b, fb in enumerate(f):
        U = nudft1(P[b], xt, yt, M)
        for iz, zz in enumerate(z):
            a, e = int(plane_ptr[iz]), int(plane_ptr[iz + 1])
            if a == e:
                continue
            Gh = dft2(kernel_samples(fb, zz, M, frame.dx, frame.dy, inv_r))
            vals = nudft2(U * Gh, rescale(vx[a:e], frame.cx, frame.Lx),
                          rescale(vy[a:e], frame.cy, frame.Ly)) / (M * M)
            out[a:e] += illumination_phase(fb, vx[a:e], vy[a:e], zz, xp) * vals
    return out


# ---------------------------------------------------------------------------
# Step 6: scaled RSD (eq. SRSD_conv with the scaled DFT of eq. RSD_scale).
# ---------------------------------------------------------------------------
def scaled_dft(x: np.ndarray, alpha: float, M: int) -> np.ndarray:
    """S[k] = sum_{n in I_N} x[n] e^{-2 pi j alpha k n / M}, k in I_M (along the
    last axis of x)."""
    N = x.shape[-1]
    E = np.exp(-2j * np.pi * alpha * np.outer(centered(N), centered(M)).astype(np.float64) / M)
    return x @ E


def relay_grid(U: np.ndarray, N: int) -> np.ndarray:
    """u[n] = M^{-2} sum_k U[k] e^{+2 pi j k.n / M} on the centred N x N window
    (the uniform relay grid that feeds the scaled RSD, obtained by NUFFT-1 and
    an inverse FFT as in the fusion for non-uniform acquisition)."""
    n = centered(N)
    return idft2_at(U, n, n)                        # [nx][ny]


def srsd_alpha(z, zref):
    return np.asarray(zref / np.asarray(z, dtype=np.float64))


def srsd(P, relay_xy, f, frame: Frame, grid, xp, alphas, inv_r=True):
    """Scaled RSD on the frustum: per plane, scaled DFT of the uniform relay
    grid u (pitch dx), times the DFT of G sampled at pitch dx / alpha, inverse
    DFT onto the N x N window; voxel (ix, iy) of plane z sits at
    c + (ix - nx//2, iy - ny//2) * d / alpha(z).  Returns V complex [Z][ny][nx]."""
    N = grid.nx
    assert grid.ny == N
    xt = rescale(relay_xy[:, 0], frame.cx, frame.Lx)
    yt = rescale(relay_xy[:, 1], frame.cy, frame.Ly)
    M = frame.M
    m = np.arange(N) - N // 2
    z = np.asarray(grid.z, dtype=np.float64)
    out = np.zeros((len(z), N, N), dtype=np.complex128)
    for b, fb in enumerate(f):
        U = nudft1(P[b], xt, yt, M)
        u = relay_grid(U, N)                         # [nx][ny]
        for iz, zz in enumerate(z):
            a = float(alphas[iz])
            S = scaled_dft(scaled_dft(u, a, M).T, a, M).T     # rows then columns
            Gh = dft2(kernel_samples(fb, zz, M, frame.dx / a, frame.dy / a, inv_r))
            Fz = idft2_at(S * Gh, m, m).T
            xs = frame.cx + m * frame.dx / a
            ys = frame.cy + m * frame.dy / a
            out[iz] += illumination_phase(fb, xs[None, :], ys[:, None], zz, xp) * Fz
    return out


def srsd_points(P, relay_xy, f, frame: Frame, N, z, alphas, plane_ptr, voxel_xy, xp, inv_r=True):
    """Fusion of the scaled RSD with NURSD-2 (eq. NURSD2_SRSD): per plane, the
    scaled spectrum S of the uniform relay grid u (as in srsd) times the DFT
    of G sampled at pitch dx / alpha, evaluated at the plane's voxel list by a
    direct NUDFT-2 in the scaled frame (period M dx / alpha around the frame
    centre).  Returns V complex [V]."""
    xt = rescale(relay_xy[:, 0], frame.cx, frame.Lx)
    yt = rescale(relay_xy[:, 1], frame.cy, frame.Ly)
    vx = np.asarray(voxel_xy[:, 0], dtype=np.float64)
    vy = np.asarray(voxel_xy[:, 1], dtype=np.float64)
    M = frame.M
    z = np.asarray(z, dtype=np.float64)
    out = np.zeros(len(vx), dtype=np.complex128)
    for b, fb in enumerate(f):
        U = nudft1(P[b], xt, yt, M)
        u = relay_grid(U, N)                         # [nx][ny]
        for iz, zz in enumerate(z):
            a0, e0 = int(plane_ptr[iz]), int(plane_ptr[iz + 1])
            if a0 == e0:
                continue
            a = float(alphas[iz])
            S = scaled_dft(scaled_dft(u, a, M).T, a, M).T
            Gh = dft2(kernel_samples(fb, zz, M, frame.dx / a, frame.dy / a, inv_r))
            vals = nudft2(S * Gh, rescale(vx[a0:e0], frame.cx, frame.Lx / a),
                          rescale(vy[a0:e0], frame.cy, frame.Ly / a)) / (M * M)
            out[a0:e0] += illumination_phase(fb, vx[a0:e0], vy[a0:e0], zz, xp) * vals
    return out


def nursd_video(P, relay_xy, f, frame: Frame, grid, xp, times, alphas=None):
    """4D light transport (eq. Video_Voxel_Freq_Offset): the coherent field of
    every voxel at each time t, V(x_v, t) = sum_b e^{+j 2 pi f_b t} W_b(x_v),
    where W_b is the single-frequency field (back-propagation and illumination
    phase) of NURSD-1, or of the scaled RSD when alphas are given.
    Returns complex [len(times)][Z][ny][nx]; the video intensity is |V|."""
    times = np.asarray(times, dtype=np.float64)
    out = np.zeros((len(times), len(grid.z), grid.ny, grid.nx), dtype=np.complex128)
    for b, fb in enumerate(f):
        if alphas is None:
            Wb = nursd_grid(P[b:b + 1], relay_xy, f[b:b + 1], frame, grid, xp)
        else:
            Wb = srsd(P[b:b + 1], relay_xy, f[b:b + 1], frame, grid, xp, alphas)
        out += np.exp(2j * np.pi * fb * times)[:, None, None, None] * Wb[None]
    return out


def nursd_grid_multi(Ps, relay_xy, f, frame: Frame, grid, xps):
    """Several illumination positions (the integral over x_p in
    eq. PF_RSD_Defn): V = sum_k NURSD-1(P_k) with the illumination phase of
    x_p,k; Ps [K][F][L] are the phasors measured under each illumination,
    xps [K][3].  Returns complex [Z][ny][nx]."""
    out = None
    for P, xp in zip(Ps, np.asarray(xps, dtype=np.float64)):
        V = nursd_grid(P, relay_xy, f, frame, grid, xp)
        out = V if out is None else out + V
    return out


def subsample_nearest(P, D):
    """Compression preprocessing of the sampling-criteria section: keep the
    relay-grid samples on the lattice of stride D per axis (the others are
    discarded) and fill every grid point from its nearest kept sample
    (Euclidean distance in grid units; ties go to the first kept sample in
    row-major order).  P: [..., ny, nx]; returns the same shape."""
    P = np.asarray(P)
    ny, nx = P.shape[-2:]
    ky, kx = np.arange(0, ny, D), np.arange(0, nx, D)
    KY, KX = np.meshgrid(ky, kx, indexing="ij")
    kept = np.stack([KY.ravel(), KX.ravel()], 1)                 # row-major order
    out = np.empty_like(P)
    for iy in range(ny):
        for ix in range(nx):
            d2 = (kept[:, 0] - iy) ** 2 + (kept[:, 1] - ix) ** 2
            sy, sx = kept[int(np.argmin(d2))]
            out[..., iy, ix] = P[..., sy, sx]
    return out


# ---------------------------------------------------------------------------
# 3D NURSD (eq. 3D_NURSD): non-planar relay surfaces.
# ---------------------------------------------------------------------------
def kernel3d_samples(f: float, M: int, dx: float, dy: float, Mz: int, dz: float) -> np.ndarray:
    """3D RSD kernel e^{+j 2 pi f r / c} (eq. 3d_rsd: no 1/r) at
    (m dx, n dy, p dz), (m, n, p) in I_M^2 x I_Mz; [p][m][n]."""
    m = centered(M).astype(np.float64)
    p = centered(Mz).astype(np.float64)
    r = np.sqrt((p * dz)[:, None, None] ** 2 + (m * dx)[None, :, None] ** 2 + (m * dy)[None, None, :] ** 2)
    return np.exp(2j * np.pi * f * r / C_LIGHT)


def nursd3d_stage1(Pb, relay_xyz, fb, frame: Frame, z0: float, dz: float, Mz: int) -> np.ndarray:
    """Stage 1 of the 3D NURSD for one frequency: the 3D type-1 NUDFT of the
    relay samples onto I_M^2 x I_Mz (z frame centred on the plane z0, pitch
    dz), times the 3D DFT of the sampled 3D kernel, inverse 3D DFT read at the
    slice z0; returned as that slice's 2D spectrum U0[kx][ky] (so the field
    at z0 is M^-2 sum_k U0[k] e^{+j k.x~})."""
    r = np.asarray(relay_xyz, dtype=np.float64)
    xt = rescale(r[:, 0], frame.cx, frame.Lx)
    yt = rescale(r[:, 1], frame.cy, frame.Ly)
    zt = 2.0 * np.pi * (r[:, 2] - z0) / (Mz * dz)
    kz = centered(Mz).astype(np.float64)
    M = frame.M
    U3 = np.stack([nudft1(np.asarray(Pb) * np.exp(-1j * k * zt), xt, yt, M) for k in kz])    # [kz][kx][ky]
    G3 = kernel3d_samples(fb, M, frame.dx, frame.dy, Mz, dz)
    Gh2 = np.stack([dft2(g) for g in G3])                                                  # [p][kx][ky]
    Dz = dft_matrix(Mz, -1.0)                                                              # [kz][p]
    Gh3 = np.tensordot(Dz, Gh2, axes=(1, 0))                                               # [kz][kx][ky]
    # inverse DFT along z read at p = 0 (the plane z0): the average over kz
    return (U3 * Gh3).sum(axis=0) / Mz


def nursd3d_grid(P, relay_xyz, f, frame: Frame, grid, xp, z0: float, dz: float, Mz: int, inv_r=True):
    """3D NURSD onto a uniform voxel grid: stage 1 (nursd3d_stage1) to the
    plane z0, then NURSD-1's plane-to-plane propagation with G = e^{+jkr}/r
    at distance z_v - z0 and the volume formation of eq. PF_RSD_Defn.
    grid.z are the voxel depths, all > z0.  Returns V complex [Z][ny][nx]."""
    mx = window_index(grid.nx, frame.q)
    my = window_index(grid.ny, frame.q)
    xs = frame.cx + mx * frame.dx
    ys = frame.cy + my * frame.dy
    z = np.asarray(grid.z, dtype=np.float64)
    out = np.zeros((len(z), grid.ny, grid.nx), dtype=np.complex128)
    for b, fb in enumerate(f):
        U0 = nursd3d_stage1(P[b], relay_xyz, fb, frame, z0, dz, Mz)
        for iz, zz in enumerate(z):
            Gh = dft2(kernel_samples(fb, zz - z0, frame.M, frame.dx, frame.dy, inv_r))
            Fz = idft2_at(U0 * Gh, mx, my).T
            out[iz] += illumination_phase(fb, xs[None, :], ys[:, None], zz, xp) * Fz
    return out


# ---------------------------------------------------------------------------
# Step 8: adjoint of the uniform-grid operator and the loss gradients.
# ---------------------------------------------------------------------------
def nursd_grid_adjoint(gV, relay_xy, f, frame: Frame, grid, xp, P=None, inv_r=True, weights=None):
    """Conjugate transpose of P -> V (nursd_grid, coherent) applied to gV
    [Z][ny][nx].  Returns grad_P [F][L] and, when P is given, the position
    gradient grad_xy [L][2] = Re sum_b conj(P_bl) dV/dx_l contracted with gV,
    i.e. for a real loss with PyTorch-style upstream gradient gV
    (dL/dRe V + j dL/dIm V): grad_P = A^H gV and
    grad_x_l = Re sum_b conj(P_bl) sum_k S_b[k] (j 2 pi kx / Lx) e^{+j k.x~_l}.
    With weights w_l (the forward map is P -> V(w P)), both gradients carry
    the factor w_l."""
    xt = rescale(relay_xy[:, 0], frame.cx, frame.Lx)
    yt = rescale(relay_xy[:, 1], frame.cy, frame.Ly)
    M = frame.M
    mx = window_index(grid.nx, frame.q)
    my = window_index(grid.ny, frame.q)
    xs = frame.cx + mx * frame.dx
    ys = frame.cy + my * frame.dy
    k = centered(M).astype(np.float64)
    Fn = len(f)
    L = relay_xy.shape[0]
    gP = np.zeros((Fn, L), dtype=np.complex128)
    gxy = np.zeros((L, 2), dtype=np.float64)
    Dx = dft_matrix(M, -1.0, rows=centered(M), cols=mx)     # [M][nx]
    Dy = dft_matrix(M, -1.0, rows=centered(M), cols=my)
    for b, fb in enumerate(f):
        S = np.zeros((M, M), dtype=np.complex128)
        for iz, zz in enumerate(grid.z):
            ph = illumination_phase(fb, xs[None, :], ys[:, None], zz, xp)
            r = (np.conj(ph) * gV[iz]).T                       # [nx][ny]
            R = Dx @ r @ Dy.T / (M * M)
            Gh = dft2(kernel_samples(fb, zz, M, frame.dx, frame.dy, inv_r))
            S += np.conj(Gh) * R
        gP[b] = nudft2(S, xt, yt)
        if P is not None:
            Sx = S * (1j * 2 * np.pi * k / frame.Lx)[:, None]
            Sy = S * (1j * 2 * np.pi * k / frame.Ly)[None, :]
            gxy[:, 0] += np.real(np.conj(P[b]) * nudft2(Sx, xt, yt))
            gxy[:, 1] += np.real(np.conj(P[b]) * nudft2(Sy, xt, yt))
    if weights is not None:
        w = np.asarray(weights, dtype=np.float64)
        gP = gP * w[None, :]
        gxy = gxy * w[:, None]
    return gP, gxy


# ---------------------------------------------------------------------------
# Physics reference: the RSD integral evaluated sample by sample (eq.
# PF_RSD_Defn with the kernel of eq. RSD_conv, i.e. filtered back-projection).
# ---------------------------------------------------------------------------
def rsd_direct(P, relay_xy, f, vox_xyz, xp, chunk: int = 4096, inv_r: bool = True):
    """V(x_v) = sum_b e^{+j k_b |x_v - x_p|} sum_l P[b][l] e^{+j k_b r_lv} / r_lv
    (no 1/r_lv when inv_r is False), relay at z = 0.  vox_xyz: [V][3];
    returns complex [V]."""
    r = np.asarray(relay_xy, dtype=np.float64)
    v = np.asarray(vox_xyz, dtype=np.float64)
    out = np.zeros(v.shape[0], dtype=np.complex128)
    for a in range(0, v.shape[0], chunk):
        e = min(v.shape[0], a + chunk)
        d = np.sqrt((v[a:e, None, 0] - r[None, :, 0]) ** 2 + (v[a:e, None, 1] - r[None, :, 1]) ** 2
                    + v[a:e, None, 2] ** 2)
        for b, fb in enumerate(f):
            Gk = np.exp(2j * np.pi * fb * d / C_LIGHT)
            if inv_r:
                Gk = Gk / d
            ph = illumination_phase(fb, v[a:e, 0], v[a:e, 1], v[a:e, 2], xp)
            out[a:e] += ph * (Gk @ np.asarray(P[b], dtype=np.complex128))
    return out


def grid_voxels(grid, frame: Frame | None = None) -> np.ndarray:
    """Voxel centres [Z*ny*nx][3] in [z][y][x] order."""
    xs = grid.x0 + np.arange(grid.nx) * grid.dx
    ys = grid.y0 + np.arange(grid.ny) * grid.dy
    Z, Y, X = np.meshgrid(np.asarray(grid.z, dtype=np.float64), ys, xs, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


# ---------------------------------------------------------------------------
# Geometry helpers (scaled-RSD section and supplement).
# ---------------------------------------------------------------------------
def frustum_volume(z: float, x_in: float, alpha: float) -> float:
    """V_F = z x_in^2 + z^2 x_in / alpha + z^3 / (3 alpha^2) (square frustum)."""
    return z * x_in ** 2 + z * z * x_in / alpha + z ** 3 / (3 * alpha ** 2)


def frustum_gain(z: float, alpha: float) -> float:
    """Delta V = V_F - V_C = (1/alpha + 1/(3 alpha^2)) z^3 for x_in = z (eq. Vol_Frustum)."""
    return (1.0 / alpha + 1.0 / (3.0 * alpha ** 2)) * z ** 3


def compression_ratio(D: float, T: int, F: int) -> float:
    """N^2 T / ((N/D)^2 2F): data saving of subsampling by D and keeping F
    complex frequency coefficients (data-savings paragraph)."""
    return D * D * T / (2.0 * F)


def lateral_resolution(lambda_c: float, z: float, aperture: float) -> float:
    """Delta x = 1.22 lambda_c z / D (eq. Focusing_Res)."""
    return 1.22 * lambda_c * z / aperture


# ---------------------------------------------------------------------------
# Whole reconstruction from histograms (steps 1-7).
# ---------------------------------------------------------------------------
def phasors_from_workload(w, hist=None):
    wl = w.wavelet
    bins, f = wavelet_bins(wl.lambda_c, wl.n_time, wl.dt, wl.n_freq, wl.bins)
    wts = phasor_weights(f, wl.lambda_c, wl.sigma_rel, wl.t0)
    h = w.hist if hist is None else hist
    return temporal_phasor(h, bins, wts), f


def frame_for_workload(w, q: int = 1) -> Frame:
    g = w.grid
    if w.mode == "points":
        return choose_frame("points", w.relay_xy, dx=g.dx, dy=g.dy, voxel_xy=w.voxel_xy, pad=w.pad, q=q)
    # the scaled RSD at voxel lists keeps the scaled RSD's frame (relay grid);
    # the 3D NURSD keeps the uniform grid's lateral frame
    mode = {"srsd_points": "srsd", "grid3d": "grid"}.get(w.mode, w.mode)
    return choose_frame(mode, w.relay_xy, x0=g.x0, y0=g.y0, dx=g.dx, dy=g.dy, nx=g.nx,
                        ny=g.ny, pad=w.pad, q=q)
