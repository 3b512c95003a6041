"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these re-types an oracle formula: each compares the oracle with a
library routine (numpy's FFT) in a special case it reduces to, with a
physically different computation (the brute-force RSD sum), with an
invariant (adjointness, Parseval, shift theorem), with finite differences,
or with values the paper prints.
"""
import math
import os

import numpy as np
import pytest

from oracle import nursd_ref as o
from workloads import scenes

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


# ------------------------------------------------------------------ step 1
def test_temporal_phasor_matches_library_fft():
    rng = np.random.default_rng(0)
    h = rng.poisson(3.0, size=(7, 64)).astype(np.float64)
    bins = np.array([1, 5, 9, 31])
    P = o.temporal_phasor(h, bins, np.ones(4))
    ref = np.fft.fft(h, axis=1)[:, bins].T
    assert rel(P, ref) < 1e-13


def test_temporal_phasor_parseval_all_bins():
    rng = np.random.default_rng(1)
    h = rng.normal(size=(3, 32))
    P = o.temporal_phasor(h, np.arange(32), np.ones(32))
    np.testing.assert_allclose((np.abs(P) ** 2).sum(0), 32 * (h ** 2).sum(1), rtol=1e-12)


def test_time_origin_is_a_physical_delay():
    # Delaying the histogram by s bins must equal moving the time origin t0 by
    # s*dt: the e^{-j 2 pi f t0} factor has the sign of a delay.
    rng = np.random.default_rng(2)
    T, dt, s = 128, 8e-12, 5
    h = rng.random((4, T))
    h[:, -s:] = 0.0
    bins, f = o.wavelet_bins(0.06, T, dt, 6, bins=np.arange(10, 16))
    a = o.temporal_phasor(np.roll(h, s, axis=1), bins, o.phasor_weights(f, 0.06, 0.2, 0.0))
    b = o.temporal_phasor(h, bins, o.phasor_weights(f, 0.06, 0.2, s * dt))
    assert rel(a, b) < 1e-12


def test_bins_of_tiny_config():
    w = scenes.config_tiny(render=False)
    bins, f = o.wavelet_bins(w.wavelet.lambda_c, w.wavelet.n_time, w.wavelet.dt, w.wavelet.n_freq)
    # f_c = c / 6 cm = 4.9965 GHz, df = 1 / (512 * 8 ps) = 244.14 MHz -> k0 = 20
    assert bins[0] == 12 and bins[-1] == 27
    with pytest.raises(ValueError):
        o.wavelet_bins(0.06, 64, 8e-12, 40)


def test_gaussian_weight_width():
    fc = o.C_LIGHT / 0.06
    w = o.phasor_weights(np.array([fc, fc + 0.2 * fc]), 0.06, 0.2, 0.0)
    np.testing.assert_allclose(np.abs(w), [1.0, math.exp(-0.5)], rtol=1e-14)


# ------------------------------------------------------------------ step 3
def _grid_points(M, n, rng, dx=0.01, c=(0.0, 0.0)):
    idx = rng.choice(M * M, size=n, replace=False)
    ix = idx // M - M // 2
    iy = idx % M - M // 2
    xy = np.stack([c[0] + ix * dx, c[1] + iy * dx], axis=1)
    return xy, ix, iy


def test_nudft1_on_grid_is_fft2():
    rng = np.random.default_rng(3)
    M = 16
    xy, ix, iy = _grid_points(M, 40, rng)
    P = rng.normal(size=40) + 1j * rng.normal(size=40)
    L = M * 0.01
    U = o.nudft1(P, o.rescale(xy[:, 0], 0, L), o.rescale(xy[:, 1], 0, L), M)
    grid = np.zeros((M, M), complex)
    grid[ix % M, iy % M] = P
    ref = np.fft.fftshift(np.fft.fft2(grid))
    assert rel(U, ref) < 1e-13


def test_nudft_pair_is_adjoint():
    rng = np.random.default_rng(4)
    M, L = 12, 30
    xt = rng.uniform(-np.pi, np.pi, L)
    yt = rng.uniform(-np.pi, np.pi, L)
    P = rng.normal(size=L) + 1j * rng.normal(size=L)
    U = rng.normal(size=(M, M)) + 1j * rng.normal(size=(M, M))
    lhs = np.vdot(U, o.nudft1(P, xt, yt, M))
    rhs = np.vdot(o.nudft2(U, xt, yt), P)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_nudft1_shift_theorem():
    rng = np.random.default_rng(5)
    M, L = 10, 20
    xt = rng.uniform(-2, 2, L)
    yt = rng.uniform(-2, 2, L)
    P = rng.normal(size=L) + 0j
    sx = 0.3
    k = o.centered(M)
    a = o.nudft1(P, xt + sx, yt, M)
    b = o.nudft1(P, xt, yt, M) * np.exp(-1j * k * sx)[:, None]
    assert rel(a, b) < 1e-13


def test_dft2_and_idft_are_library_transforms():
    rng = np.random.default_rng(6)
    M = 16
    g = rng.normal(size=(M, M)) + 1j * rng.normal(size=(M, M))
    ref = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(g)))
    assert rel(o.dft2(g), ref) < 1e-13
    m = o.centered(M)
    back = o.idft2_at(ref, m, m)
    assert rel(back, g) < 1e-13


# ------------------------------------------------------------------ steps 4-7
def _on_grid_case(rng, M=32, n=8, L=25, dx=0.02, F=3, zs=(0.15, 0.31)):
    """Relays on grid points inside the central half, voxels the n x n window."""
    c = n // 2
    x0 = -c * dx
    grid = scenes.Grid(x0=x0, y0=x0, dx=dx, dy=dx, nx=n, ny=n, z=np.array(zs))
    idx = rng.choice(n * n, size=L, replace=False)
    xy = np.stack([x0 + (idx % n) * dx, x0 + (idx // n) * dx], axis=1)
    frame = o.Frame(M, dx, dx, 0.0, 0.0)
    f = np.array([2.1e9, 3.3e9, 4.4e9])[:F]
    P = rng.normal(size=(F, L)) + 1j * rng.normal(size=(F, L))
    return grid, xy, frame, f, P


def test_on_grid_nursd_equals_brute_force_rsd():
    # Discrete convolution theorem with zero padding: for relays on the grid
    # the FFT-based propagation is exactly the RSD sum over relay samples.
    rng = np.random.default_rng(7)
    grid, xy, frame, f, P = _on_grid_case(rng)
    xp = np.array([0.05, -0.02, 0.0])
    V = o.nursd_grid(P, xy, f, frame, grid, xp)
    ref = o.rsd_direct(P, xy, f, o.grid_voxels(grid), xp).reshape(V.shape)
    assert rel(V, ref) < 1e-11


def test_points_mode_on_grid_voxels_equals_grid_mode():
    rng = np.random.default_rng(8)
    grid, xy, frame, f, P = _on_grid_case(rng)
    xyz = o.grid_voxels(grid)
    nv = grid.nx * grid.ny
    sel = rng.choice(len(xyz), 40, replace=False)
    sel.sort()
    V = o.nursd_grid(P, xy, f, frame, grid, np.zeros(3)).ravel()[sel]
    zi = sel // nv
    ptr = np.searchsorted(zi, np.arange(len(grid.z) + 1))
    Vp = o.nursd_points(P, xy, f, frame, grid.z, ptr, xyz[sel, :2], np.zeros(3))
    assert rel(Vp, V) < 1e-11


def test_point_scatterer_focuses_at_its_voxel():
    # A rendered point scatterer, phasor-transformed and back-propagated, must
    # peak at its own voxel (signs of the temporal and spatial phases).
    w = scenes.config_tiny(render=False)
    g = w.grid
    s = np.array([[g.x0 + 21 * g.dx, g.y0 + 9 * g.dy, g.z[13]]])
    h = scenes.render_transients(w.relay_xy, s, np.ones(1), w.xp, w.wavelet.n_time,
                                 w.wavelet.dt, w.wavelet.t0)
    P, f = o.phasors_from_workload(w, h)
    fr = o.frame_for_workload(w)
    I = np.abs(o.nursd_grid(P, w.relay_xy.astype(np.float64), f, fr, g, w.xp))
    iz, iy, ix = np.unravel_index(I.argmax(), I.shape)
    assert abs(ix - 21) <= 1 and abs(iy - 9) <= 1 and abs(iz - 13) <= 1


def test_video_peak_follows_a_measurement_delay():
    # 4D light transport: at a point scatterer's voxel the video peaks near
    # t = 0; delaying every histogram by d bins (the returns arrive d dt
    # later) moves that peak to t = +d dt.  Fixes the sign of the time phase
    # relative to the temporal transform.
    w = scenes.config_tiny(render=False)
    g = w.grid
    s = np.array([[g.x0 + 21 * g.dx, g.y0 + 9 * g.dy, g.z[13]]])
    h = scenes.render_transients(w.relay_xy, s, np.ones(1), w.xp, w.wavelet.n_time,
                                 w.wavelet.dt, w.wavelet.t0)
    d = 20
    fr = o.frame_for_workload(w)
    sub = scenes.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny, g.z[13:14])
    times = np.arange(-30, 51) * 10e-12
    peaks = []
    for hh in (h, np.roll(h, d, axis=1)):
        P, f = o.phasors_from_workload(w, hh)
        Vt = o.nursd_video(P, w.relay_xy.astype(np.float64), f, fr, sub, w.xp, times)
        peaks.append(times[np.argmax(np.abs(Vt[:, 0, 9, 21]))])
    assert abs(peaks[0]) <= 20e-12
    assert abs(peaks[1] - peaks[0] - d * w.wavelet.dt) <= 10e-12


def test_lateral_psf_width_loose():
    # Lateral resolution 1.22 lambda z / D (eq. Focusing_Res): the lateral
    # half-maximum width of a focused point is within a loose band of it.
    n = 64
    dx = 0.01
    x0 = -n // 2 * dx
    relay = np.stack(np.meshgrid(np.arange(-24, 24) * 0.02, np.arange(-24, 24) * 0.02), -1).reshape(-1, 2)
    D = 0.96
    zs = 0.8
    f = np.array([o.C_LIGHT / 0.06])
    s = np.array([0.0, 0.0, zs])
    r = np.sqrt(((relay - s[:2]) ** 2).sum(1) + zs ** 2)
    P = np.exp(-2j * np.pi * f[0] * (r + zs) / o.C_LIGHT)[None, :]   # ideal phasors of s
    vx = x0 + np.arange(n) * dx
    vox = np.stack([vx, np.zeros(n), np.full(n, zs)], 1)
    I = np.abs(o.rsd_direct(P, relay, f, vox, np.zeros(3)))
    above = vx[I >= I.max() / 2]
    width = above.max() - above.min()
    expect = o.lateral_resolution(0.06, zs, D)
    assert 0.5 * expect < width < 1.5 * expect


def test_off_grid_gap_is_small_when_oversampled():
    # Off the grid, NURSD is the trigonometric interpolant of the sampled
    # kernel, not the RSD sum; with a pitch well below lambda/2 the two agree
    # closely (the paper calls the difference negligible).  Reported, loose.
    rng = np.random.default_rng(9)
    dx = 0.004
    n = 16
    grid = scenes.Grid(x0=-8 * dx, y0=-8 * dx, dx=dx, dy=dx, nx=n, ny=n, z=np.array([0.3]))
    xy = rng.uniform(-7 * dx, 7 * dx, size=(30, 2))
    frame = o.Frame(64, dx, dx, 0.0, 0.0)
    f = np.array([3e9])
    P = rng.normal(size=(1, 30)) + 0j
    V = o.nursd_grid(P, xy, f, frame, grid, np.zeros(3))
    ref = o.rsd_direct(P, xy, f, o.grid_voxels(grid), np.zeros(3)).reshape(V.shape)
    assert rel(V, ref) < 0.05


# ------------------------------------------------------------------ step 6
def test_scaled_dft_special_cases_are_library_ffts():
    rng = np.random.default_rng(10)
    N, M = 8, 16
    x = rng.normal(size=N) + 1j * rng.normal(size=N)
    # alpha = 1: a zero-padded DFT of length M
    pad = np.zeros(M, complex)
    pad[o.centered(N) % M] = x
    ref1 = np.fft.fftshift(np.fft.fft(pad))
    assert rel(o.scaled_dft(x, 1.0, M), ref1) < 1e-13
    # alpha = 1/2: every output is a bin of a zero-padded DFT of length 2M
    pad2 = np.zeros(2 * M, complex)
    pad2[o.centered(N) % (2 * M)] = x
    F2 = np.fft.fft(pad2)
    ref2 = F2[o.centered(M) % (2 * M)]
    assert rel(o.scaled_dft(x, 0.5, M), ref2) < 1e-13


def test_srsd_alpha_one_is_nursd_on_grid():
    rng = np.random.default_rng(11)
    grid, xy, frame, f, P = _on_grid_case(rng)
    xp = np.array([0.0, 0.01, 0.0])
    V1 = o.nursd_grid(P, xy, f, frame, grid, xp)
    Vs = o.srsd(P, xy, f, frame, grid, xp, np.ones(len(grid.z)))
    assert rel(Vs, V1) < 1e-11


def test_srsd_double_scale_equals_brute_force_rsd():
    # With alpha = 2 the output pitch dx / alpha is half the relay pitch, so the
    # relays n dx sit on the output grid and the scaled RSD must equal the RSD
    # sum at voxels c + m' dx / alpha (M >= 4N keeps the convolution linear).
    # alpha > 1 is outside the range the paper uses but the identity holds
    # for any alpha, which pins the scaled DFT and the stretched kernel.
    rng = np.random.default_rng(12)
    grid, xy, frame, f, P = _on_grid_case(rng, M=32, n=8, L=20)
    xp = np.array([0.02, 0.0, 0.0])
    alpha = 2.0
    Vs = o.srsd(P, xy, f, frame, grid, xp, np.full(len(grid.z), alpha))
    m = np.arange(grid.nx) - grid.nx // 2
    xs = m * grid.dx / alpha
    Z, Y, X = np.meshgrid(grid.z, xs, xs, indexing="ij")
    vox = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    ref = o.rsd_direct(P, xy, f, vox, xp).reshape(Vs.shape)
    assert rel(Vs, ref) < 1e-11


def test_srsd_equals_nursd_in_stretched_frame():
    # Second route: the scaled RSD equals NURSD-1 in a frame of pitch dx/alpha
    # fed with the uniform relay grid u at its physical positions n dx.
    rng = np.random.default_rng(13)
    grid, xy, frame, f, P = _on_grid_case(rng, M=32, n=8, L=20, zs=(0.2,))
    alpha = 0.7
    xp = np.zeros(3)
    Vs = o.srsd(P, xy, f, frame, grid, xp, np.array([alpha]))
    n = grid.nx
    m = np.arange(n) - n // 2
    u = [o.relay_grid(o.nudft1(P[b], o.rescale(xy[:, 0], 0, frame.Lx),
                                o.rescale(xy[:, 1], 0, frame.Ly), frame.M), n) for b in range(len(f))]
    X, Y = np.meshgrid(m * grid.dx, m * grid.dx, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], 1)
    Pu = np.stack([ub.ravel() for ub in u])
    d2 = grid.dx / alpha
    g2 = scenes.Grid(x0=-(n // 2) * d2, y0=-(n // 2) * d2, dx=d2, dy=d2, nx=n, ny=n, z=grid.z)
    fr2 = o.Frame(frame.M, d2, d2, 0.0, 0.0)
    V2 = o.nursd_grid(Pu, pts, f, fr2, g2, xp)
    assert rel(Vs, V2) < 1e-11


def test_srsd_points_at_scaled_grid_voxels_equals_srsd():
    # Voxel lists placed on each plane's scaled grid c + m dx / alpha must
    # reproduce the uniform scaled RSD there (planes with different alpha).
    rng = np.random.default_rng(21)
    grid, xy, frame, f, P = _on_grid_case(rng, M=32, n=8, L=20)
    xy = xy + rng.uniform(-0.006, 0.006, size=xy.shape)        # off grid
    xp = np.array([0.01, -0.02, 0.0])
    alphas = np.array([0.8, 0.45])
    Vs = o.srsd(P, xy, f, frame, grid, xp, alphas)               # [Z][ny][nx]
    m = np.arange(grid.nx) - grid.nx // 2
    pick = [rng.choice(grid.nx * grid.ny, 11, replace=False), rng.choice(grid.nx * grid.ny, 7, replace=False)]
    vox, ref = [], []
    for iz, a in enumerate(alphas):
        iy, ix = np.divmod(pick[iz], grid.nx)
        vox.append(np.stack([frame.cx + m[ix] * grid.dx / a, frame.cy + m[iy] * grid.dy / a], 1))
        ref.append(Vs[iz, iy, ix])
    ptr = np.array([0, len(pick[0]), len(pick[0]) + len(pick[1])])
    V = o.srsd_points(P, xy, f, frame, grid.nx, grid.z, alphas, ptr, np.concatenate(vox), xp)
    assert rel(V, np.concatenate(ref)) < 1e-11


def test_srsd_points_equals_nursd_points_in_stretched_frame():
    # Independent route at arbitrary voxels: NURSD-3 in a frame of pitch
    # dx / alpha, fed with the uniform relay grid u at its physical positions.
    rng = np.random.default_rng(22)
    grid, xy, frame, f, P = _on_grid_case(rng, M=32, n=8, L=20, zs=(0.2,))
    xy = xy + rng.uniform(-0.006, 0.006, size=xy.shape)
    alpha = 0.6
    xp = np.array([0.0, 0.01, 0.0])
    n = grid.nx
    half = 0.5 * frame.M * grid.dx / alpha
    vox = rng.uniform(-0.45 * half, 0.45 * half, size=(13, 2))
    ptr = np.array([0, len(vox)])
    V = o.srsd_points(P, xy, f, frame, n, grid.z, np.array([alpha]), ptr, vox, xp)
    m = np.arange(n) - n // 2
    u = [o.relay_grid(o.nudft1(P[b], o.rescale(xy[:, 0], 0, frame.Lx),
                                o.rescale(xy[:, 1], 0, frame.Ly), frame.M), n) for b in range(len(f))]
    X, Y = np.meshgrid(m * grid.dx, m * grid.dx, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], 1)
    Pu = np.stack([ub.ravel() for ub in u])
    d2 = grid.dx / alpha
    fr2 = o.Frame(frame.M, d2, d2, 0.0, 0.0)
    ref = o.nursd_points(Pu, pts, f, fr2, grid.z, ptr, vox, xp)
    assert rel(V, ref) < 1e-11


def test_multi_illumination_on_grid_equals_brute_force_rsd():
    # Several laser positions, each with its own phasors: on-grid relays make
    # the FFT route exact, so the sum must equal the brute-force RSD sums with
    # each position's illumination phase.
    rng = np.random.default_rng(31)
    grid, xy, frame, f, P = _on_grid_case(rng, F=2)
    Ps = [P, rng.normal(size=P.shape) + 1j * rng.normal(size=P.shape)]
    xps = np.array([[0.05, -0.02, 0.0], [-0.07, 0.04, 0.01]])
    V = o.nursd_grid_multi(Ps, xy, f, frame, grid, xps)
    vox = o.grid_voxels(grid)
    ref = sum(o.rsd_direct(Pk, xy, f, vox, xk) for Pk, xk in zip(Ps, xps)).reshape(V.shape)
    assert rel(V, ref) < 1e-11


@pytest.mark.parametrize("D,ny,nx", [(1, 5, 7), (2, 5, 7), (3, 8, 9), (4, 9, 6)])
def test_subsample_nearest_is_the_separable_lattice_rule(D, ny, nx):
    # On a product lattice the nearest kept point is found axis by axis: round
    # i / D to the nearest integer (halves down), clamp to the last kept index.
    rng = np.random.default_rng(32)
    P = rng.normal(size=(2, ny, nx)) + 1j * rng.normal(size=(2, ny, nx))
    out = o.subsample_nearest(P, D)

    def near(i, n):
        q = np.floor((i + (D - 1) / 2) / D).astype(int) * D   # ties to the lower kept index
        return np.minimum(q, (n - 1) // D * D)
    sy, sx = near(np.arange(ny), ny), near(np.arange(nx), nx)
    assert np.array_equal(out, P[:, sy[:, None], sx[None, :]])
    assert np.array_equal(out[:, ::D, ::D], P[:, ::D, ::D])     # kept samples unchanged


def test_3d_stage1_on_lattice_equals_brute_force():
    # Relays on the 3D lattice (grid points in x, y; z0 + q dz in depth) and
    # field points in the central window: the 3D FFT route of stage 1 is the
    # discrete 3D convolution, so it must equal the direct sum of the 3D RSD
    # kernel over the samples (eq. 3d_rsd) to round-off.
    rng = np.random.default_rng(41)
    M, n, dx, Mz, dz, L = 32, 16, 0.02, 8, 0.015, 30
    z0 = 0.1
    frame = o.Frame(M, dx, dx, 0.0, 0.0)
    c = np.arange(n) - n // 2
    ix, iy = rng.integers(0, n, L), rng.integers(0, n, L)
    q = rng.integers(-Mz // 4, Mz // 4 + 1, L)
    xyz = np.stack([c[ix] * dx, c[iy] * dx, z0 + q * dz], 1)
    P = rng.normal(size=L) + 1j * rng.normal(size=L)
    fb = 3.1e9
    U0 = o.nursd3d_stage1(P, xyz, fb, frame, z0, dz, Mz)
    F0 = o.idft2_at(U0, c, c)                                    # [x][y] on the window
    X, Y = np.meshgrid(c * dx, c * dx, indexing="ij")
    r = np.sqrt((X[..., None] - xyz[:, 0]) ** 2 + (Y[..., None] - xyz[:, 1]) ** 2 + (z0 - xyz[:, 2]) ** 2)
    ref = (np.exp(2j * np.pi * fb * r / o.C_LIGHT) * P).sum(-1)
    assert rel(F0, ref) < 1e-11


def test_3d_nursd_of_a_flat_wall_on_the_lattice_matches_two_stage_brute_force():
    # A flat wall on the lattice (all z_l = z0 - 2 dz): stage 1 (brute force, as
    # pinned above) gives the field on the plane z0 on the window; stage 2 is
    # NURSD-1 of that field from grid positions at z0.  The full 3D NURSD must
    # equal that composition when the field is confined to the window.
    rng = np.random.default_rng(42)
    M, n, dx, Mz, dz, L = 32, 16, 0.02, 8, 0.015, 25
    z0 = 0.1
    frame = o.Frame(M, dx, dx, 0.0, 0.0)
    c = np.arange(n) - n // 2
    g = scenes.Grid(x0=c[0] * dx, y0=c[0] * dx, dx=dx, dy=dx, nx=n, ny=n, z=np.array([0.25, 0.4]))
    idx = rng.choice(n * n, L, replace=False)
    xyz = np.stack([c[idx % n] * dx, c[idx // n] * dx, np.full(L, z0 - 2 * dz)], 1)
    f = np.array([2.2e9, 3.0e9])
    P = rng.normal(size=(2, L)) + 1j * rng.normal(size=(2, L))
    xp = np.array([0.01, 0.0, 0.0])
    V = o.nursd3d_grid(P, xyz, f, frame, g, xp, z0, dz, Mz)
    # composition: the stage-1 spectrum, evaluated as a field on the whole
    # period grid, fed as phasors at those grid points into NURSD-1 (z - z0)
    m = o.centered(M)
    X, Y = np.meshgrid(m * dx, m * dx, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], 1)
    F0 = np.stack([o.idft2_at(o.nursd3d_stage1(P[b], xyz, f[b], frame, z0, dz, Mz), m, m).ravel()
                   for b in range(2)])
    gs = scenes.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny, g.z - z0)
    ref = o.nursd_grid(F0, pts, f, frame, gs, xp - np.array([0, 0, z0]))
    assert rel(V, ref) < 1e-10


# ------------------------------------------------------------------ step 8
def _adj_case(rng):
    grid, xy, frame, f, P = _on_grid_case(rng, M=16, n=6, L=12, zs=(0.12, 0.2))
    xy = xy + rng.uniform(-0.004, 0.004, size=xy.shape)       # off grid
    return grid, xy, frame, f, P


def test_adjoint_dot_product():
    rng = np.random.default_rng(14)
    grid, xy, frame, f, P = _adj_case(rng)
    xp = np.array([0.01, 0.0, 0.0])
    V = o.nursd_grid(P, xy, f, frame, grid, xp)
    gV = rng.normal(size=V.shape) + 1j * rng.normal(size=V.shape)
    gP, _ = o.nursd_grid_adjoint(gV, xy, f, frame, grid, xp)
    lhs = np.vdot(gV, V)
    rhs = np.vdot(gP, P)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(15)
    grid, xy, frame, f, P = _adj_case(rng)
    xp = np.zeros(3)
    Vt = o.nursd_grid(P, xy + 0.002, f, frame, grid, xp)

    def loss(Pv, xyv):
        return float(np.sum(np.abs(o.nursd_grid(Pv, xyv, f, frame, grid, xp) - Vt) ** 2))

    V = o.nursd_grid(P, xy, f, frame, grid, xp)
    gP, gxy = o.nursd_grid_adjoint(2 * (V - Vt), xy, f, frame, grid, xp, P)
    h = 1e-7
    for l, ax in [(0, 0), (3, 1), (7, 0), (11, 1)]:
        e = np.zeros_like(xy)
        e[l, ax] = h
        fd = (loss(P, xy + e) - loss(P, xy - e)) / (2 * h)
        assert abs(fd - gxy[l, ax]) < 1e-5 * max(1.0, abs(gxy).max())
    for b, l in [(0, 2), (2, 5)]:
        e = np.zeros_like(P)
        e[b, l] = 1e-6
        fr = (loss(P + e, xy) - loss(P - e, xy)) / 2e-6
        fi = (loss(P + 1j * e, xy) - loss(P - 1j * e, xy)) / 2e-6
        assert abs(fr - gP[b, l].real) < 1e-5 * abs(gP).max()
        assert abs(fi - gP[b, l].imag) < 1e-5 * abs(gP).max()


# ------------------------------------------------------------------ helpers
def _golden(name):
    rows = [l.split() for l in open(os.path.join(GOLD, name)) if l.strip() and not l.startswith("#")]
    return [[float(v) for v in r] for r in rows]


def test_frustum_worked_example():
    for alpha, z, vc, vf, dv, pct in _golden("frustum_example.txt"):
        assert round(z ** 3) == vc
        assert round(o.frustum_volume(z, z, alpha)) == vf
        assert round(o.frustum_gain(z, alpha)) == dv
        assert round(100 * o.frustum_gain(z, alpha) / z ** 3) == pct


def test_data_savings_worked_example():
    for D, T, F, ratio in _golden("data_savings.txt"):
        assert round(o.compression_ratio(D, T, F)) == ratio


def test_frame_rule_for_the_workloads():
    expect = {"tiny": 64, "spad": 512, "diff": 256, "frustum_points": 512, "srsd": 512}
    for w in [scenes.config_tiny(False), scenes.config_spad(False), scenes.config_diff(False),
              scenes.config_frustum_points(False), scenes.config_srsd(False)]:
        assert o.frame_for_workload(w).M == expect[w.name]
