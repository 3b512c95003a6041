"""GPU adjoint and gradients (through the C ABI and torch.autograd) against
the FP64 oracle adjoint, the dot-product identity and finite differences."""
import numpy as np
import pytest
import torch

from oracle import nursd_ref as o
from workloads import scenes

pytestmark = pytest.mark.gpu
TOL = 1e-4


def rel(a, b):
    r = float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))
    print(f"  rel-L2 {r:.3e}", flush=True)
    return r


def adj_case(seed=11, n=20, L=200, nz=3, F=3):
    rng = np.random.default_rng(seed)
    dx = 0.02
    g = scenes.Grid(x0=-0.19, y0=-0.17, dx=dx, dy=dx, nx=n, ny=n - 3, z=np.linspace(0.25, 0.5, nz))
    xy = np.stack([rng.uniform(-0.17, 0.17, L), rng.uniform(-0.15, 0.12, L)], 1).astype(np.float32)
    wl = scenes.Wavelet(lambda_c=0.06, n_time=512, dt=8e-12, t0=0.0, n_freq=F, bins=np.array([13, 19, 24])[:F])
    w = scenes.Workload("adj", xy, np.array([0.02, -0.01, 0.0]), wl, g)
    P = (rng.normal(size=(F, L)) + 1j * rng.normal(size=(F, L))).astype(np.complex64)
    gV = (rng.normal(size=(nz, n - 3, n)) + 1j * rng.normal(size=(nz, n - 3, n))).astype(np.complex64)
    return w, P, gV


def plan_for(w, device, **kw):
    from paper_2501_05244_amd.api import plan_from_workload
    return plan_from_workload(w, device, **kw)


@pytest.mark.parametrize("chunks", [(0, 0), (2, 1)])
def test_adjoint_matches_oracle(device, chunks):
    print("case: adjoint small", chunks, flush=True)
    w, P, gV = adj_case()
    plan = plan_for(w, device, freq_chunk=chunks[0], plane_chunk=chunks[1])
    gP, gxy = plan.adjoint(torch.from_numpy(gV).to(device), torch.from_numpy(P).to(device))
    fr = o.frame_for_workload(w)
    _, f = o.wavelet_bins(0.06, 512, 8e-12, 3, w.wavelet.bins)
    rgP, rgxy = o.nursd_grid_adjoint(gV.astype(np.complex128), w.relay_xy.astype(np.float64), f, fr, w.grid, w.xp,
                                     P.astype(np.complex128))
    assert rel(gP.cpu().numpy(), rgP) < TOL
    assert rel(gxy.cpu().numpy(), rgxy) < TOL


def test_autograd_function(device):
    from paper_2501_05244_amd.autograd import nursd
    w, P, _ = adj_case(seed=12)
    plan = plan_for(w, device)
    fr = o.frame_for_workload(w)
    _, f = o.wavelet_bins(0.06, 512, 8e-12, 3, w.wavelet.bins)
    xy64 = w.relay_xy.astype(np.float64)
    Vt = o.nursd_grid(P.astype(np.complex128), xy64 + 0.002, f, fr, w.grid, w.xp)
    Pt = torch.from_numpy(P).to(device).requires_grad_(True)
    xyt = torch.from_numpy(w.relay_xy).to(device).requires_grad_(True)
    V = nursd(Pt, xyt, plan)
    loss = (V - torch.from_numpy(Vt.astype(np.complex64)).to(device)).abs().pow(2).sum()
    loss.backward()
    Vref = o.nursd_grid(P.astype(np.complex128), xy64, f, fr, w.grid, w.xp)
    rgP, rgxy = o.nursd_grid_adjoint(2 * (Vref - Vt), xy64, f, fr, w.grid, w.xp, P.astype(np.complex128))
    assert rel(Pt.grad.cpu().numpy(), rgP) < TOL
    assert rel(xyt.grad.cpu().numpy(), rgxy) < TOL


def test_dot_product_identity_full_diff_config(device):
    """<A P, gV> = <P, A^H gV> at the full differentiation-config size
    (16,384 relays, 48 frequencies, 128x128x64 voxels)."""
    print("case: adjoint dot product full size", flush=True)
    w = scenes.config_diff(render=False)
    plan = plan_for(w, device)
    g = torch.Generator(device="cpu").manual_seed(5)
    P = torch.randn((plan.F, plan.L), dtype=torch.complex64, generator=g).to(device)
    gV = torch.randn((len(w.grid.z), w.grid.ny, w.grid.nx), dtype=torch.complex64, generator=g).to(device)
    V, _ = plan.forward_phasor(P, intensity=False)
    gP, _ = plan.adjoint(gV)
    lhs = torch.vdot(gV.flatten().to(torch.complex128), V.flatten().to(torch.complex128))
    rhs = torch.vdot(gP.flatten().to(torch.complex128), P.flatten().to(torch.complex128))
    assert abs(complex(lhs - rhs)) < 1e-4 * abs(complex(lhs))


@pytest.mark.slow
def test_diff_config_reduced_copy_vs_oracle(device):
    """Differentiation workload with the same relays and voxel grid but 4
    frequencies and 8 planes: GPU gradients vs the FP64 oracle adjoint, and
    central finite differences (h = 1e-4 m) of the GPU loss."""
    print("case: diff reduced copy", flush=True)
    from paper_2501_05244_amd.autograd import nursd
    w = scenes.config_diff(render=True)
    w.wavelet.bins = np.array([30, 37, 44, 51])
    w.grid.z = w.grid.z[::8]
    plan = plan_for(w, device)
    wl = w.wavelet
    bins, f = o.wavelet_bins(wl.lambda_c, wl.n_time, wl.dt, 4, wl.bins)
    P = np.ascontiguousarray(o.temporal_phasor(w.hist, bins, o.phasor_weights(f, wl.lambda_c, 0.2, 0.0))
                             .astype(np.complex64))
    fr = o.frame_for_workload(w)
    xy64 = w.relay_xy.astype(np.float64)
    Vt = o.nursd_grid(P.astype(np.complex128), xy64 + w.extra["delta"].astype(np.float64), f, fr, w.grid, w.xp)
    Vt32 = torch.from_numpy(Vt.astype(np.complex64)).to(device)
    Pt = torch.from_numpy(P).to(device).requires_grad_(True)
    xyt = torch.from_numpy(w.relay_xy).to(device).requires_grad_(True)
    loss = (nursd(Pt, xyt, plan) - Vt32).abs().pow(2).sum()
    loss.backward()
    Vref = o.nursd_grid(P.astype(np.complex128), xy64, f, fr, w.grid, w.xp)
    rgP, rgxy = o.nursd_grid_adjoint(2 * (Vref - Vt), xy64, f, fr, w.grid, w.xp, P.astype(np.complex128))
    assert rel(Pt.grad.cpu().numpy(), rgP) < TOL
    assert rel(xyt.grad.cpu().numpy(), rgxy) < TOL
    # central differences of the GPU loss on 8 seeded samples, loose (FP32 loss)
    h = 1e-4
    rng = np.random.default_rng(32)
    gx = xyt.grad.cpu().numpy()
    for l in rng.choice(w.relay_xy.shape[0], 8, replace=False):
        for ax in (0, 1):
            vals = []
            for sgn in (1, -1):
                xy = w.relay_xy.copy()
                xy[l, ax] += sgn * h
                plan.set_points(torch.from_numpy(xy).to(device))
                V, _ = plan.forward_phasor(torch.from_numpy(P).to(device), intensity=False)
                vals.append(float((V.to(torch.complex128) - Vt32.to(torch.complex128)).abs().pow(2).sum()))
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - gx[l, ax]) < 0.05 * abs(gx).max()
