"""Seeded synthetic NLOS workloads (input generation only).

This module renders the inputs that both the GPU path and the FP64 oracle
consume: relay-sample positions, transient histograms of point/patch scenes,
voxel geometries and per-plane voxel lists.  It contains none of the
reconstruction arithmetic (no phasor transform, no NUFFT, no RSD kernel).

Light-transport model used for rendering (the measurement the paper's
phasor-field section starts from, a three-bounce impulse response): for a
scatterer s with albedo a, laser spot x_p and relay sample x_c,
    r1 = |x_p - s|, r2 = |s - x_c|, tau = (r1 + r2) / c,
    amplitude a / (r1^2 r2^2),
deposited with a linear split between bins floor((tau - t0)/dt) and the next,
modulo T.  Poisson noise (optional) scales the histograms so the largest bin
equals the stated peak and then draws counts with numpy's PCG64.

Shapes follow the paper's setups: relay extents of 1-2 m, central wavelength
4-8 cm, picosecond bins, 32x32 SPAD arrays imaged obliquely.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

C_LIGHT = 299_792_458.0


@dataclasses.dataclass
class Wavelet:
    lambda_c: float          # central wavelength [m]
    n_time: int              # T
    dt: float                # bin width [s]
    t0: float                # time of bin 0 [s]
    n_freq: int              # F
    sigma_rel: float = 0.2   # sigma_f / f_c
    bins: np.ndarray | None = None   # explicit DFT bins (overrides the centred band)


@dataclasses.dataclass
class Grid:
    """Uniform voxel grid: voxel (ix, iy) centre = (x0 + ix*dx, y0 + iy*dy)."""
    x0: float
    y0: float
    dx: float
    dy: float
    nx: int
    ny: int
    z: np.ndarray            # plane depths [m], float64 [Z]


@dataclasses.dataclass
class Workload:
    name: str
    relay_xy: np.ndarray     # float32 [L][2]
    xp: np.ndarray           # float64 [3], laser spot
    wavelet: Wavelet
    grid: Grid
    hist: np.ndarray | None = None        # float32 [L][T]
    scatterers: np.ndarray | None = None  # float64 [S][3]
    albedo: np.ndarray | None = None      # float64 [S]
    mode: str = "grid"                    # "grid" | "points" | "srsd" | "srsd_points" | "grid3d"
    plane_ptr: np.ndarray | None = None   # int32 [Z+1] (points mode)
    voxel_xy: np.ndarray | None = None    # float32 [V][2] (points mode)
    zref: float = 0.0                     # srsd: alpha(z) = zref / z
    pad: float = 2.0
    extra: dict = dataclasses.field(default_factory=dict)


def cell_centres(lo: float, hi: float, n: int) -> np.ndarray:
    step = (hi - lo) / n
    return lo + step * (np.arange(n) + 0.5)


# ---------------------------------------------------------------- relay layouts
def relay_uniform(n: int, half: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-half, half, size=(n, 2)).astype(np.float32)


def relay_spad_oblique(seed: int, pixels: int = 32, poses: int = 8, extent: float = 2.0,
                       jitter: float = 1e-3, keystone: float = 0.3) -> np.ndarray:
    """A pixels x pixels SPAD array imaged obliquely onto the relay wall at
    poses x poses scan positions tiling an extent x extent wall.  Each pose maps
    the pixel grid through a plane-to-plane homography with a keystone (the
    footprint narrows along one axis, as for a camera tilted ~45 degrees off the
    wall normal), then adds N(0, jitter) positional noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cell = extent / poses
    s = (np.arange(pixels) + 0.5) / pixels - 0.5
    S, Tt = np.meshgrid(s, s, indexing="xy")
    denom = 1.0 + keystone * Tt
    u = S / denom
    v = Tt / denom
    # scale the footprint so that its widest extent stays inside the pose cell
    span = max(u.max() - u.min(), v.max() - v.min())
    scale = 0.96 * cell / span
    u = (u - 0.5 * (u.max() + u.min())) * scale
    v = (v - 0.5 * (v.max() + v.min())) * scale
    out = []
    for j in range(poses):
        for i in range(poses):
            cx = -extent / 2 + cell * (i + 0.5)
            cy = -extent / 2 + cell * (j + 0.5)
            out.append(np.stack([u.ravel() + cx, v.ravel() + cy], axis=1))
    xy = np.concatenate(out, axis=0)
    xy += rng.normal(0.0, jitter, size=xy.shape)
    lim = extent / 2 - 1e-3
    np.clip(xy, -lim, lim, out=xy)
    return xy.astype(np.float32)


# ---------------------------------------------------------------- scenes
def scatter_points(n: int, lateral: float, zlo: float, zhi: float, seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    xy = rng.uniform(-lateral, lateral, size=(n, 2))
    z = rng.uniform(zlo, zhi, size=(n, 1))
    alb = rng.uniform(0.5, 1.0, size=n)
    return np.concatenate([xy, z], axis=1), alb


def patch(centre, size: float, tilt_deg: float = 0.0, step: float = 0.01):
    """Square patch of side `size`, discretised at `step` (cell centres), tilted
    about the x axis by tilt_deg; total albedo 1 spread evenly."""
    n = max(1, int(round(size / step)))
    c = cell_centres(-size / 2, size / 2, n)
    U, V = np.meshgrid(c, c, indexing="xy")
    t = math.radians(tilt_deg)
    x = centre[0] + U
    y = centre[1] + V * math.cos(t)
    z = centre[2] + V * math.sin(t)
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    return pts, np.full(pts.shape[0], 1.0 / pts.shape[0])


def render_transients(relay_xy: np.ndarray, scat: np.ndarray, albedo: np.ndarray,
                      xp: np.ndarray, n_time: int, dt: float, t0: float,
                      chunk: int = 1024) -> np.ndarray:
    """Three-bounce transients H[l][t] (float32), relay at z = 0."""
    L = relay_xy.shape[0]
    out = np.empty((L, n_time), dtype=np.float32)
    scat = np.asarray(scat, dtype=np.float64)
    r1 = np.linalg.norm(scat - np.asarray(xp, dtype=np.float64)[None, :], axis=1)  # [S]
    for a in range(0, L, chunk):
        b = min(L, a + chunk)
        rc = relay_xy[a:b].astype(np.float64)
        dxy = scat[None, :, :2] - rc[:, None, :]
        r2 = np.sqrt((dxy ** 2).sum(-1) + scat[None, :, 2] ** 2)       # [l][S]
        tau = (r1[None, :] + r2) / C_LIGHT
        pos = (tau - t0) / dt
        i0 = np.floor(pos)
        frac = pos - i0
        amp = albedo[None, :] / (r1[None, :] ** 2 * r2 ** 2)
        i0 = np.mod(i0.astype(np.int64), n_time)
        i1 = np.mod(i0 + 1, n_time)
        rows = np.arange(b - a, dtype=np.int64)[:, None] * n_time
        idx = np.concatenate([(rows + i0).ravel(), (rows + i1).ravel()])
        w = np.concatenate([(amp * (1.0 - frac)).ravel(), (amp * frac).ravel()])
        h = np.bincount(idx, weights=w, minlength=(b - a) * n_time)
        out[a:b] = h.reshape(b - a, n_time).astype(np.float32)
    return out


def poisson_counts(hist: np.ndarray, peak: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = hist.astype(np.float64) * (peak / float(hist.max()))
    return rng.poisson(lam).astype(np.float32)


# ---------------------------------------------------------------- configurations
def config_tiny(render: bool = True) -> Workload:
    """1,024 random relay samples over 1x1 m, 512 bins at 8 ps, 3 scatterers,
    Poisson peak 100, 6 cm wavelength (16 frequencies), 32x32x32 voxels."""
    relay = relay_uniform(1024, 0.5, seed=1)
    scat, alb = scatter_points(3, 0.4, 0.5, 1.5, seed=2)
    wl = Wavelet(lambda_c=0.06, n_time=512, dt=8e-12, t0=0.0, n_freq=16)
    n = 32
    grid = Grid(x0=-0.5 + 0.5 / n, y0=-0.5 + 0.5 / n, dx=1.0 / n, dy=1.0 / n, nx=n, ny=n,
                z=cell_centres(0.5, 1.5, 32))
    w = Workload("tiny", relay, np.zeros(3), wl, grid, scatterers=scat, albedo=alb)
    if render:
        h = render_transients(relay, scat, alb, w.xp, wl.n_time, wl.dt, wl.t0)
        w.hist = poisson_counts(h, 100.0, seed=3)
    return w


def spad_scene():
    pts, alb = scatter_points(200, 0.8, 1.0, 2.5, seed=12)
    p1, a1 = patch((-0.4, 0.3, 1.5), 0.4, 0.0)
    p2, a2 = patch((0.45, -0.35, 2.2), 0.4, 30.0)
    return np.concatenate([pts, p1, p2]), np.concatenate([alb, a1, a2])


def config_spad(render: bool = True) -> Workload:
    """65,536 relay samples (32x32 SPAD array, 64 oblique poses, 1 mm jitter)
    over 2x2 m; 4,096 bins at 4 ps; 200 points + 2 patches; 6 cm wavelength
    with 96 frequencies; 256x256x128 voxels over [-1,1]^2 x [1,3] m."""
    relay = relay_spad_oblique(seed=11)
    scat, alb = spad_scene()
    wl = Wavelet(lambda_c=0.06, n_time=4096, dt=4e-12, t0=1.8 / C_LIGHT, n_freq=96)
    n = 256
    grid = Grid(x0=-1.0 + 1.0 / n, y0=-1.0 + 1.0 / n, dx=2.0 / n, dy=2.0 / n, nx=n, ny=n,
                z=cell_centres(1.0, 3.0, 128))
    w = Workload("spad", relay, np.zeros(3), wl, grid, scatterers=scat, albedo=alb)
    if render:
        w.hist = render_transients(relay, scat, alb, w.xp, wl.n_time, wl.dt, wl.t0)
    return w


def config_frustum_points(render: bool = True, planes: int = 64, per_side: int = 128) -> Workload:
    """Same input as config_spad, reconstructed at per-plane voxel lists: 64
    planes over [1,4] m, per plane a 128x128 lattice at pitch 15.625 mm * z/1 m,
    each point jittered uniformly by +-pitch/2 (a perspective frustum)."""
    w = config_spad(render)
    rng = np.random.Generator(np.random.PCG64(21))
    z = cell_centres(1.0, 4.0, planes)
    xy = []
    ptr = [0]
    for zz in z:
        p = 0.015625 * zz
        c = (np.arange(per_side) - (per_side - 1) / 2.0) * p
        X, Y = np.meshgrid(c, c, indexing="xy")
        pts = np.stack([X.ravel(), Y.ravel()], axis=1)
        pts += rng.uniform(-p / 2, p / 2, size=pts.shape)
        xy.append(pts)
        ptr.append(ptr[-1] + pts.shape[0])
    w.name = "frustum_points"
    w.mode = "points"
    w.voxel_xy = np.concatenate(xy).astype(np.float32)
    w.plane_ptr = np.asarray(ptr, dtype=np.int32)
    # FFT pitch 10 m / 512 (about half the shortest wavelength); no uniform voxels
    w.grid = Grid(x0=0.0, y0=0.0, dx=10.0 / 512, dy=10.0 / 512, nx=0, ny=0, z=z)
    return w


def config_srsd(render: bool = True) -> Workload:
    """Same input as config_spad reconstructed by the scaled RSD: 256x256
    samples per plane at pitch 7.8125 mm * z / 1 m, 128 planes over [1,4] m."""
    w = config_spad(render)
    n = 256
    w.name = "srsd"
    w.mode = "srsd"
    w.grid = Grid(x0=-1.0 + 1.0 / n, y0=-1.0 + 1.0 / n, dx=2.0 / n, dy=2.0 / n, nx=n, ny=n,
                  z=cell_centres(1.0, 4.0, 128))
    w.zref = 1.0
    return w


def config_srsd_points(render: bool = True, planes: int = 64, per_side: int = 128) -> Workload:
    """Scaled RSD frustum at voxel lists: the scaled-RSD relay grid (256x256
    over [-1,1]^2, zref = 1 m) evaluated at the jittered perspective lattices
    of config_frustum_points (64 planes over [1,4] m, 128x128 points per plane
    at pitch 15.625 mm * z/1 m): 1,048,576 voxels."""
    fr = config_frustum_points(render, planes, per_side)
    w = config_srsd(False)
    w.hist = fr.hist
    w.name = "srsd_points"
    w.mode = "srsd_points"
    w.plane_ptr = fr.plane_ptr
    w.voxel_xy = fr.voxel_xy
    w.grid = Grid(w.grid.x0, w.grid.y0, w.grid.dx, w.grid.dy, w.grid.nx, w.grid.ny, z=fr.grid.z)
    return w


def nonplanar_wall(xy: np.ndarray, amp: float) -> np.ndarray:
    """Depth of a curved relay wall at lateral positions xy: a smooth bump and
    ripple, |z| <= amp."""
    x, y = xy[:, 0].astype(np.float64), xy[:, 1].astype(np.float64)
    return (amp * (0.6 * np.cos(0.5 * np.pi * x) * np.cos(0.5 * np.pi * y) - 0.4 * np.sin(2.3 * x + 1.1 * y))
            ).astype(np.float32)


def config_nonplanar(render: bool = False) -> Workload:
    """3D NURSD at SPAD scale: the 65,536 oblique SPAD samples of config_spad
    on a curved wall (depth within +-5 cm), intermediate plane 6 cm in front,
    3D grid depth pitch 2 cm, 96 frequencies, 256x256x128 voxels over
    [-1,1]^2 x [1,3] m.  Histograms are not rendered (phasors are inputs)."""
    w = config_spad(render=False)
    w.name = "nonplanar"
    w.mode = "grid3d"
    w.extra = {"relay_z": nonplanar_wall(w.relay_xy, 0.05), "z_mid": 0.06, "dz3": 0.02}
    return w


def config_diff(render: bool = True) -> Workload:
    """16,384 random relay samples over 1x1 m, 1,024 bins at 8 ps, 10
    scatterers, 6 cm wavelength (48 frequencies), 128x128x64 voxels; relay
    calibration offsets N(0, 2 mm) (seed 32) in extra['delta']."""
    relay = relay_uniform(16384, 0.5, seed=31)
    scat, alb = scatter_points(10, 0.4, 0.5, 1.5, seed=33)
    wl = Wavelet(lambda_c=0.06, n_time=1024, dt=8e-12, t0=0.0, n_freq=48)
    n = 128
    grid = Grid(x0=-0.5 + 0.5 / n, y0=-0.5 + 0.5 / n, dx=1.0 / n, dy=1.0 / n, nx=n, ny=n,
                z=cell_centres(0.5, 1.5, 64))
    w = Workload("diff", relay, np.zeros(3), wl, grid, scatterers=scat, albedo=alb)
    rng = np.random.Generator(np.random.PCG64(32))
    w.extra["delta"] = rng.normal(0.0, 2e-3, size=relay.shape).astype(np.float32)
    if render:
        w.hist = render_transients(relay, scat, alb, w.xp, wl.n_time, wl.dt, wl.t0)
    return w


def config_batch(render: bool = True, n_scenes: int = 64, seed: int = 41) -> list[Workload]:
    """64 scenes of uneven size: relay counts log-uniform in [2048, 65536],
    N in {64,96,128,192,256} with Z = N/2, F uniform in 16..128 (capped so the
    band stays inside (0, T/2)), wavelength uniform in [4,8] cm, pitch
    7.8125 mm, T = 2048 at 4 ps, 1-20 scatterers."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    dx = 0.0078125
    for s in range(n_scenes):
        L = int(round(math.exp(rng.uniform(math.log(2048), math.log(65536)))))
        n = int(rng.choice([64, 96, 128, 192, 256]))
        F = int(rng.integers(16, 129))
        lam = float(rng.uniform(0.04, 0.08))
        T, dt = 2048, 4e-12
        k0 = round((C_LIGHT / lam) * T * dt)
        F = min(F, 2 * (k0 - 1))
        half = n * dx / 2
        nsc = int(rng.integers(1, 21))
        rseed = int(rng.integers(0, 2 ** 31))
        relay = relay_uniform(L, half * 0.999, seed=rseed)
        zlo = 0.5
        zhi = zlo + n * dx
        scat, alb = scatter_points(nsc, 0.8 * half, zlo, zhi, seed=rseed + 1)
        wl = Wavelet(lambda_c=lam, n_time=T, dt=dt, t0=0.0, n_freq=F)
        grid = Grid(x0=-half + dx / 2, y0=-half + dx / 2, dx=dx, dy=dx, nx=n, ny=n,
                    z=cell_centres(zlo, zhi, n // 2))
        w = Workload(f"batch{s}", relay, np.zeros(3), wl, grid, scatterers=scat, albedo=alb)
        if render:
            w.hist = render_transients(relay, scat, alb, w.xp, T, dt, wl.t0)
        out.append(w)
    return out


def tone_histograms(n_relay: int, n_time: int, bins, seed: int) -> np.ndarray:
    """Histograms that are sums of sinusoids at the given DFT bins:
    H[l][t] = sum_j Re(A_lj e^{+2 pi i b_j t / T}) with A_lj complex normal
    (seeded), float32 [L][T].  Their temporal spectrum vanishes outside the
    bins +-b_j, which restricts a reconstruction to those frequencies while
    the input keeps the shape of a full measurement."""
    rng = np.random.Generator(np.random.PCG64(seed))
    bins = np.asarray(bins, dtype=np.int64)
    A = rng.normal(size=(n_relay, len(bins))) + 1j * rng.normal(size=(n_relay, len(bins)))
    t = np.arange(n_time, dtype=np.float64)
    E = np.exp(2j * np.pi * np.outer(bins, t) / n_time)          # [J][T]
    return np.ascontiguousarray((A @ E).real.astype(np.float32))


def work_units(w: Workload) -> int:
    """Voxel-frequency propagations of one reconstruction."""
    if w.mode in ("points", "srsd_points"):
        nvox = int(w.plane_ptr[-1])
    else:
        nvox = w.grid.nx * w.grid.ny * len(w.grid.z)
    nf = w.wavelet.n_freq if w.wavelet.bins is None else len(w.wavelet.bins)
    return nvox * nf
