"""GPU parity of the NURSD forward path (through the C ABI) against the FP64
oracle.  Tolerance: relative L2 <= 1e-4 on the complex volume and on the
intensity (the target of the method's FP32 implementation); stage tests
use tighter bounds derived from FP32 round-off of each stage."""
import numpy as np
import pytest
import torch

from oracle import nursd_ref as o
from workloads import scenes

pytestmark = pytest.mark.gpu

TOL = 1e-4


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    r = float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
    print(f"  rel-L2 {r:.3e}", flush=True)
    return r


def to_fft_order(Uc, M):
    k = o.centered(M)
    out = np.zeros_like(Uc)
    out[..., (k % M)[:, None], (k % M)[None, :]] = Uc
    return out


def plan_for(w, device, **kw):
    from paper_2501_05244_amd.api import plan_from_workload
    return plan_from_workload(w, device, **kw)


@pytest.fixture(scope="module")
def tiny():
    return scenes.config_tiny()


def test_frame_matches_oracle(device, tiny):
    plan = plan_for(tiny, device)
    fr = o.frame_for_workload(tiny)
    assert plan.info["M"] == fr.M and plan.info["Mf"] == 2 * fr.M
    assert abs(plan.info["cx"] - fr.cx) < 1e-12 and abs(plan.info["cy"] - fr.cy) < 1e-12
    assert plan.info["dx"] == fr.dx and plan.info["dy"] == fr.dy


def test_phasor_tiny(device, tiny):
    print("case: phasor tiny", flush=True)
    plan = plan_for(tiny, device)
    P = plan.phasor(torch.from_numpy(tiny.hist).to(device)).cpu().numpy()
    Pref, _ = o.phasors_from_workload(tiny)
    assert rel(P, Pref) < 2e-6


@pytest.mark.parametrize("T,F,offset", [(2048, 37, 0), (4096, 130, 0), (2048, 16, 2)])
def test_phasor_wavefront_ragged(device, T, F, offset):
    """Phasor stage at T = 2048 and 4096 (one wavefront per histogram), with
    a relay count that leaves a partial group of 16 and F above 128; offset 2
    floats starts the rows on an 8-byte (not 16-byte) boundary, which takes
    the block-level transform instead."""
    print(f"case: phasor T={T} F={F} offset={offset}", flush=True)
    w = scenes.config_tiny(render=False)
    L = 1000
    w.relay_xy = w.relay_xy[:L]
    w.wavelet.n_time = T
    w.wavelet.dt = 4e-12
    w.wavelet.n_freq = F
    w.wavelet.t0 = 1.3e-9
    rng = np.random.default_rng(7)
    hist = rng.poisson(3.0, size=(L, T)).astype(np.float32)
    plan = plan_for(w, device)
    buf = torch.zeros(offset + L * T, dtype=torch.float32, device=device)
    buf[offset:] = torch.from_numpy(hist.ravel()).to(device)
    P = plan.phasor(buf[offset:].view(L, T)).cpu().numpy()
    Pref, _ = o.phasors_from_workload(w, hist)
    assert rel(P, Pref) < 2e-6


def test_phasor_rejects_misaligned_histograms(device, tiny):
    """A histogram pointer off an 8-byte boundary is refused on the host."""
    plan = plan_for(tiny, device)
    L, T = tiny.hist.shape
    buf = torch.zeros(1 + L * T, dtype=torch.float32, device=device)
    with pytest.raises(RuntimeError, match="aligned"):
        plan.phasor(buf[1:].view(L, T))


def test_spectrum_tiny(device, tiny):
    print("case: spectrum tiny", flush=True)
    plan = plan_for(tiny, device)
    Pref, _ = o.phasors_from_workload(tiny)
    P32 = np.ascontiguousarray(Pref.astype(np.complex64))
    U = plan.spectrum(torch.from_numpy(P32).to(device)).cpu().numpy()
    fr = o.frame_for_workload(tiny)
    xy = tiny.relay_xy.astype(np.float64)
    Uc = o.nudft1(P32.astype(np.complex128), o.rescale(xy[:, 0], fr.cx, fr.Lx), o.rescale(xy[:, 1], fr.cy, fr.Ly),
                  fr.M) / fr.M ** 2
    assert rel(U, to_fft_order(Uc, fr.M)) < 5e-6


def test_forward_tiny_from_histograms(device, tiny):
    print("case: forward tiny", flush=True)
    plan = plan_for(tiny, device)
    V, I = plan.forward_hist(torch.from_numpy(tiny.hist).to(device))
    Pref, f = o.phasors_from_workload(tiny)
    fr = o.frame_for_workload(tiny)
    Vref = o.nursd_grid(Pref, tiny.relay_xy.astype(np.float64), f, fr, tiny.grid, tiny.xp)
    assert rel(V.cpu().numpy(), Vref) < TOL
    assert rel(I.cpu().numpy(), np.abs(Vref)) < TOL


def test_forward_is_bitwise_reproducible(device, tiny):
    plan = plan_for(tiny, device)
    h = torch.from_numpy(tiny.hist).to(device)
    V1, _ = plan.forward_hist(h)
    V2, _ = plan.forward_hist(h)
    assert torch.equal(torch.view_as_real(V1), torch.view_as_real(V2))


def ragged_case(seed=5, nx=20, ny=13, nz=5, L=300, F=3):
    rng = np.random.default_rng(seed)
    dx = 0.02
    g = scenes.Grid(x0=-0.19, y0=-0.13, dx=dx, dy=dx, nx=nx, ny=ny, z=np.linspace(0.21, 0.6, nz))
    xy = np.stack([rng.uniform(-0.18, 0.18, L), rng.uniform(-0.12, 0.12, L)], 1).astype(np.float32)
    wl = scenes.Wavelet(lambda_c=0.06, n_time=512, dt=8e-12, t0=0.0, n_freq=F, bins=np.array([13, 19, 26]))
    w = scenes.Workload("ragged", xy, np.array([0.01, -0.02, 0.0]), wl, g)
    P = (rng.normal(size=(F, L)) + 1j * rng.normal(size=(F, L))).astype(np.complex64)
    return w, P


@pytest.mark.parametrize("chunks", [(0, 0), (2, 2), (1, 3)])
def test_forward_ragged_grid_and_chunks(device, chunks):
    print("case: ragged", chunks, flush=True)
    w, P = ragged_case()
    plan = plan_for(w, device, freq_chunk=chunks[0], plane_chunk=chunks[1])
    V, I = plan.forward_phasor(torch.from_numpy(P).to(device))
    fr = o.frame_for_workload(w)
    assert plan.info["M"] == fr.M
    _, f = o.wavelet_bins(w.wavelet.lambda_c, w.wavelet.n_time, w.wavelet.dt, 3, w.wavelet.bins)
    Vref = o.nursd_grid(P.astype(np.complex128), w.relay_xy.astype(np.float64), f, fr, w.grid, w.xp)
    assert rel(V.cpu().numpy(), Vref) < TOL
    assert rel(I.cpu().numpy(), np.abs(Vref)) < TOL


@pytest.mark.parametrize("L,F,nz,nx,ny", [(1, 1, 1, 1, 1), (1, 2, 2, 3, 1), (7, 1, 1, 33, 2), (65, 3, 1, 1, 40)])
def test_forward_degenerate_sizes(device, L, F, nz, nx, ny):
    """A single relay, a single frequency or plane, and one-pixel-wide
    windows: every tile of every pass is ragged (transform sizes 64 and 128)."""
    print("case: degenerate", L, F, nz, nx, ny, flush=True)
    rng = np.random.default_rng(L * 100 + nx)
    dx = 0.02
    g = scenes.Grid(x0=-0.19, y0=-0.13, dx=dx, dy=dx, nx=nx, ny=ny, z=np.linspace(0.25, 0.5, nz))
    xy = np.stack([rng.uniform(-0.18, 0.18, L), rng.uniform(-0.12, 0.12, L)], 1).astype(np.float32)
    wl = scenes.Wavelet(lambda_c=0.06, n_time=512, dt=8e-12, t0=0.0, n_freq=F, bins=np.array([13, 19, 26])[:F])
    w = scenes.Workload("degenerate", xy, np.array([0.01, -0.02, 0.0]), wl, g)
    P = (rng.normal(size=(F, L)) + 1j * rng.normal(size=(F, L))).astype(np.complex64)
    plan = plan_for(w, device)
    fr = o.frame_for_workload(w)
    assert plan.info["M"] == fr.M
    V, I = plan.forward_phasor(torch.from_numpy(P).to(device))
    _, f = o.wavelet_bins(0.06, 512, 8e-12, F, w.wavelet.bins)
    Vref = o.nursd_grid(P.astype(np.complex128), xy.astype(np.float64), f, fr, g, w.xp)
    assert V.shape == Vref.shape
    assert rel(V.cpu().numpy(), Vref) < TOL
    assert rel(I.cpu().numpy(), np.abs(Vref)) < TOL


@pytest.mark.parametrize("L,nx,ny,M", [(1, 200, 1, 512), (2, 260, 3, 1024)])
def test_forward_degenerate_large_frames(device, L, nx, ny, M):
    """One or two relays on 512- and 1024-point frames with 9 frequencies:
    nearly every spreading band is empty, the last group of the 8-frequency
    spreading tile holds one frequency, and the x transform of the fine rows
    is the register-resident one."""
    print("case: degenerate large frame", L, nx, ny, M, flush=True)
    rng = np.random.default_rng(L)
    dx = 0.02
    F = 9
    g = scenes.Grid(x0=-dx * nx / 2, y0=-0.01, dx=dx, dy=dx, nx=nx, ny=ny, z=np.array([0.4]))
    xy = np.stack([rng.uniform(-0.18, 0.18, L), rng.uniform(-0.12, 0.12, L)], 1).astype(np.float32)
    wl = scenes.Wavelet(lambda_c=0.06, n_time=512, dt=8e-12, t0=0.0, n_freq=F, bins=np.arange(12, 12 + F))
    w = scenes.Workload("degenerate_large", xy, np.array([0.01, -0.02, 0.0]), wl, g)
    P = (rng.normal(size=(F, L)) + 1j * rng.normal(size=(F, L))).astype(np.complex64)
    plan = plan_for(w, device)
    fr = o.frame_for_workload(w)
    assert plan.info["M"] == fr.M == M
    V, I = plan.forward_phasor(torch.from_numpy(P).to(device))
    _, f = o.wavelet_bins(0.06, 512, 8e-12, F, w.wavelet.bins)
    Vref = o.nursd_grid(P.astype(np.complex128), xy.astype(np.float64), f, fr, g, w.xp)
    assert V.shape == Vref.shape
    assert rel(V.cpu().numpy(), Vref) < TOL
    assert rel(I.cpu().numpy(), np.abs(Vref)) < TOL


def test_forward_incoherent(device):
    w, P = ragged_case(seed=6)
    plan = plan_for(w, device, coherent=False)
    _, I = plan.forward_phasor(torch.from_numpy(P).to(device), vol=False)
    fr = o.frame_for_workload(w)
    _, f = o.wavelet_bins(w.wavelet.lambda_c, w.wavelet.n_time, w.wavelet.dt, 3, w.wavelet.bins)
    Iref = o.nursd_grid(P.astype(np.complex128), w.relay_xy.astype(np.float64), f, fr, w.grid, w.xp,
                        coherent=False)
    assert rel(I.cpu().numpy(), Iref) < TOL


def test_on_grid_relays_match_brute_force_rsd(device):
    # relays on grid points: the FP32 GPU result must match the RSD sum itself
    rng = np.random.default_rng(7)
    n, dx, L = 16, 0.02, 60
    g = scenes.Grid(x0=-8 * dx, y0=-8 * dx, dx=dx, dy=dx, nx=n, ny=n, z=np.array([0.25, 0.4, 0.55]))
    idx = rng.choice(n * n, L, replace=False)
    xy = np.stack([g.x0 + (idx % n) * dx, g.y0 + (idx // n) * dx], 1).astype(np.float32)
    wl = scenes.Wavelet(lambda_c=0.06, n_time=512, dt=8e-12, t0=0.0, n_freq=2, bins=np.array([15, 22]))
    w = scenes.Workload("ongrid", xy, np.zeros(3), wl, g)
    P = (rng.normal(size=(2, L)) + 1j * rng.normal(size=(2, L))).astype(np.complex64)
    plan = plan_for(w, device)
    V, _ = plan.forward_phasor(torch.from_numpy(P).to(device))
    _, f = o.wavelet_bins(0.06, 512, 8e-12, 2, wl.bins)
    ref = o.rsd_direct(P.astype(np.complex128), xy.astype(np.float64), f, o.grid_voxels(g), w.xp)
    assert rel(V.cpu().numpy().ravel(), ref) < TOL


def test_errors_are_reported(device):
    w, P = ragged_case()
    from paper_2501_05244_amd.api import Plan
    xy = torch.from_numpy(w.relay_xy).to(device)
    with pytest.raises(RuntimeError, match="GEOMETRY"):
        Plan(xy, lambda_c=0.06, n_time=512, dt=8e-12, t0=0.0, n_freq=3, z=[0.2, -0.1], x0=-0.19, y0=-0.13,
             dx=0.02, dy=0.02, nx=20, ny=13)
    with pytest.raises(RuntimeError, match="ARG"):
        Plan(xy, lambda_c=0.06, n_time=512, dt=8e-12, t0=0.0, n_freq=3, z=[0.2], bins=[0, 3, 4], x0=-0.19,
             y0=-0.13, dx=0.02, dy=0.02, nx=20, ny=13)
    with pytest.raises(RuntimeError, match="UNSUPPORTED_SIZE"):
        Plan(xy, lambda_c=0.06, n_time=512, dt=8e-12, t0=0.0, n_freq=3, z=[0.2], x0=-0.19, y0=-0.13,
             dx=0.02, dy=0.02, nx=20, ny=13, M=96)
    with pytest.raises(RuntimeError, match="ARG"):
        Plan(xy[:0], lambda_c=0.06, n_time=512, dt=8e-12, t0=0.0, n_freq=3, z=[0.2], x0=-0.19, y0=-0.13,
             dx=0.02, dy=0.02, nx=20, ny=13)
    far = xy.clone()
    far[0, 0] = 5.0
    with pytest.raises(RuntimeError, match="GEOMETRY"):
        Plan(far, lambda_c=0.06, n_time=512, dt=8e-12, t0=0.0, n_freq=3, z=[0.2], x0=-0.19, y0=-0.13,
             dx=0.02, dy=0.02, nx=20, ny=13, M=64)


@pytest.mark.slow
def test_diff_config_forward_full(device):
    """16,384 relays, 48 frequencies, 128x128x64 voxels: full-volume parity."""
    print("case: diff full forward", flush=True)
    w = scenes.config_diff()
    plan = plan_for(w, device)
    V, I = plan.forward_hist(torch.from_numpy(w.hist).to(device))
    Pref, f = o.phasors_from_workload(w)
    fr = o.frame_for_workload(w)
    Vref = o.nursd_grid(Pref, w.relay_xy.astype(np.float64), f, fr, w.grid, w.xp)
    assert rel(V.cpu().numpy(), Vref) < TOL
    assert rel(I.cpu().numpy(), np.abs(Vref)) < TOL
