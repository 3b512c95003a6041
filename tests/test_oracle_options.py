"""Pins of the oracle's plan options: the upsampled frame (internal pitch =
voxel pitch / q), the kernel amplitude switch (G = e^{jkr}/r or e^{jkr}) and
per-sample weights.

As in test_oracle_pins, none of these re-types an oracle formula: the
upsampled frame and the kernel switch are checked against the brute-force
RSD sum (exact for relays on the frame's grid, by the discrete convolution
theorem with zero padding), the weights against the unweighted operator on
a subset of relays, the adjoint by the dot-product identity and finite
differences, and the frame rule against the sizes it must produce.
"""
import numpy as np
import pytest

from oracle import nursd_ref as o
from workloads import scenes


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _fine_grid_case(rng, q, n=8, vdx=0.04, L=40, F=2, zs=(0.2, 0.35), nz_off=0):
    """Voxels at pitch vdx; relays on the frame grid of pitch vdx / q, inside
    the voxel window (so every relay-voxel offset is a multiple of the grid
    pitch and lies within half a period)."""
    x0 = -(n // 2) * vdx
    grid = scenes.Grid(x0=x0, y0=x0, dx=vdx, dy=vdx, nx=n, ny=n, z=np.array(zs))
    fr = o.choose_frame("grid", np.zeros((1, 2)), x0=x0, y0=x0, dx=vdx, dy=vdx, nx=n, ny=n, q=q)
    span = (n - 1) * q                 # grid points covering the voxel window
    first = -(n * q) // 2              # grid index of voxel 0
    idx = rng.choice((span + 1) ** 2, L, replace=False)
    gx = first + idx % (span + 1)
    gy = first + idx // (span + 1)
    xy = np.stack([fr.cx + gx * fr.dx, fr.cy + gy * fr.dy], axis=1)
    f = np.array([2.3e9, 3.9e9])[:F]
    P = rng.normal(size=(F, L)) + 1j * rng.normal(size=(F, L))
    return grid, fr, xy, f, P


@pytest.mark.parametrize("q", [2, 3])
def test_upsampled_frame_on_grid_equals_brute_force_rsd(q):
    # Relays on the q-times finer grid: NURSD on the upsampled frame is the
    # RSD sum exactly, at every voxel of the (coarser) window.  A wrong
    # window index, centre or pitch moves the voxels and fails this.
    rng = np.random.default_rng(40 + q)
    grid, fr, xy, f, P = _fine_grid_case(rng, q)
    assert fr.q == q and abs(fr.dx - grid.dx / q) < 1e-15
    xp = np.array([0.03, -0.01, 0.0])
    V = o.nursd_grid(P, xy, f, fr, grid, xp)
    ref = o.rsd_direct(P, xy, f, o.grid_voxels(grid), xp).reshape(V.shape)
    assert rel(V, ref) < 1e-11


def test_upsampled_frame_size_rule():
    # M >= pad * q * max(nx, ny): the 32^3 tiny workload needs M = 64 at q = 1,
    # 128 at q = 2 and 256 at q = 4 (its relays lie inside the window).
    w = scenes.config_tiny(render=False)
    assert [o.frame_for_workload(w, q).M for q in (1, 2, 4)] == [64, 128, 256]
    fr = o.frame_for_workload(w, 2)
    # voxel (0, 0) is the grid point x0, y0
    assert abs(fr.cx + o.window_index(w.grid.nx, 2)[0] * fr.dx - w.grid.x0) < 1e-12


def test_unit_amplitude_kernel_on_grid_equals_brute_force_rsd():
    # The kernel switch without 1/r: the same on-grid identity against the
    # brute-force sum of unit-amplitude phases.
    rng = np.random.default_rng(45)
    grid, fr, xy, f, P = _fine_grid_case(rng, 1)
    xp = np.array([0.0, 0.02, 0.0])
    V = o.nursd_grid(P, xy, f, fr, grid, xp, inv_r=False)
    ref = o.rsd_direct(P, xy, f, o.grid_voxels(grid), xp, inv_r=False).reshape(V.shape)
    assert rel(V, ref) < 1e-11
    # and it differs from the 1/r kernel by far more than round-off
    assert rel(o.nursd_grid(P, xy, f, fr, grid, xp), ref) > 0.1


def test_zero_one_weights_select_relays():
    # Weights of 0 and 1 must reproduce the unweighted operator on the
    # relays of weight 1 (a wrong index or a weight on the wrong axis fails).
    rng = np.random.default_rng(46)
    grid, fr, xy, f, P = _fine_grid_case(rng, 2)
    keep = rng.random(xy.shape[0]) < 0.5
    w = keep.astype(np.float64)
    V = o.nursd_grid(P, xy, f, fr, grid, np.zeros(3), weights=w)
    ref = o.nursd_grid(P[:, keep], xy[keep], f, fr, grid, np.zeros(3))
    assert rel(V, ref) < 1e-12


def _off_grid(rng, q):
    grid, fr, xy, f, P = _fine_grid_case(rng, q, n=6, vdx=0.03, L=12, zs=(0.12, 0.2))
    xy = xy + rng.uniform(-0.004, 0.004, size=xy.shape)
    return grid, fr, xy, f, P


@pytest.mark.parametrize("q", [1, 2])
def test_adjoint_dot_product_with_options(q):
    # <A(w P), v> = <P, A^H v> with the upsampled frame, the unit-amplitude
    # kernel and per-sample weights all in play.
    rng = np.random.default_rng(47 + q)
    grid, fr, xy, f, P = _off_grid(rng, q)
    w = rng.uniform(0.2, 1.5, size=xy.shape[0])
    xp = np.array([0.01, 0.0, 0.0])
    V = o.nursd_grid(P, xy, f, fr, grid, xp, inv_r=False, weights=w)
    gV = rng.normal(size=V.shape) + 1j * rng.normal(size=V.shape)
    gP, _ = o.nursd_grid_adjoint(gV, xy, f, fr, grid, xp, inv_r=False, weights=w)
    lhs = np.vdot(gV, V)
    assert abs(lhs - np.vdot(gP, P)) < 1e-12 * abs(lhs)


def test_weighted_gradients_match_finite_differences():
    rng = np.random.default_rng(49)
    grid, fr, xy, f, P = _off_grid(rng, 2)
    w = rng.uniform(0.2, 1.5, size=xy.shape[0])
    xp = np.zeros(3)
    Vt = o.nursd_grid(P, xy + 0.002, f, fr, grid, xp, weights=w)

    def loss(Pv, xyv):
        return float(np.sum(np.abs(o.nursd_grid(Pv, xyv, f, fr, grid, xp, weights=w) - Vt) ** 2))

    V = o.nursd_grid(P, xy, f, fr, grid, xp, weights=w)
    gP, gxy = o.nursd_grid_adjoint(2 * (V - Vt), xy, f, fr, grid, xp, P, weights=w)
    h = 1e-7
    for l, ax in [(0, 0), (5, 1), (11, 0)]:
        e = np.zeros_like(xy)
        e[l, ax] = h
        fd = (loss(P, xy + e) - loss(P, xy - e)) / (2 * h)
        assert abs(fd - gxy[l, ax]) < 1e-5 * max(1.0, abs(gxy).max())
    for b, l in [(0, 2), (1, 7)]:
        e = np.zeros_like(P)
        e[b, l] = 1e-6
        fr_ = (loss(P + e, xy) - loss(P - e, xy)) / 2e-6
        fi = (loss(P + 1j * e, xy) - loss(P - 1j * e, xy)) / 2e-6
        assert abs(fr_ - gP[b, l].real) < 1e-5 * abs(gP).max()
        assert abs(fi - gP[b, l].imag) < 1e-5 * abs(gP).max()


def test_off_grid_method_gap_shrinks_with_upsampling():
    # Off the grid NURSD interpolates the sampled kernel; the paper calls the
    # difference from the RSD sum negligible when relays are oversampled.  At
    # the tiny workload's 31.25 mm pitch (above lambda_min / 2) the gap is
    # visible, and sampling the frame twice as finely must shrink it.
    w = scenes.config_tiny(render=False)
    rng = np.random.default_rng(50)
    xy = w.relay_xy[:256].astype(np.float64)
    bins, f = o.wavelet_bins(w.wavelet.lambda_c, w.wavelet.n_time, w.wavelet.dt, w.wavelet.n_freq)
    sel = [0, 8, 15]
    P = rng.normal(size=(3, 256)) + 1j * rng.normal(size=(3, 256))
    g = w.grid
    sub = scenes.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny, g.z[[4, 20]])
    ref = o.rsd_direct(P, xy, f[sel], o.grid_voxels(sub), w.xp).reshape(2, g.ny, g.nx)
    gaps = [rel(o.nursd_grid(P, xy, f[sel], o.frame_for_workload(w, q), sub, w.xp), ref) for q in (1, 2)]
    assert gaps[0] > 1e-3
    assert gaps[1] < 0.5 * gaps[0]
