"""Spreading tiles (the blur step of the NUFFT section) through the C ABI:
every tile the plans accept (band rows x frequencies per workgroup) must give
bit-identical results, since each fine-grid cell takes its samples in the
same order whatever the tile; the tiles differ only in how the walk, the x
transform and fine y share out the work (one-row bands, several rows, a
partial last frequency group, the register and the LDS transforms).  Tiles
that do not fit a plan's fine grid are rejected.  The default tile itself is
checked against the oracle by the other parity tests."""
import numpy as np
import pytest
import torch

from workloads import scenes

pytestmark = pytest.mark.gpu

TILES = (108, 116, 208, 404, 802, 1601)


def case(seed, L=1500, F=12):
    rng = np.random.default_rng(seed)
    dx = 0.02
    g = scenes.Grid(x0=-0.31, y0=-0.27, dx=dx, dy=dx, nx=32, ny=28, z=np.array([0.35, 0.8]))
    xy = np.stack([rng.uniform(-0.5, 0.5, L), rng.uniform(-0.45, 0.45, L)], 1).astype(np.float32)
    wl = scenes.Wavelet(lambda_c=0.06, n_time=512, dt=8e-12, t0=0.0, n_freq=F)
    w = scenes.Workload("tiles", xy, np.array([0.0, 0.05, 0.0]), wl, g)
    P = (rng.normal(size=(F, L)) + 1j * rng.normal(size=(F, L))).astype(np.complex64)
    return w, P


@pytest.mark.parametrize("M", [128, 256, 512])
def test_every_tile_gives_identical_results(device, M):
    from paper_2501_05244_amd.api import plan_from_workload
    w, P = case(seed=M)
    Pd = torch.from_numpy(P).to(device)
    ref = None
    for tile in (0,) + TILES:
        print(f"case: M {M} spreading tile {tile}", flush=True)
        plan = plan_from_workload(w, device, M=M, spread_tile=tile)
        assert plan.info["M"] == M
        V, _ = plan.forward_phasor(Pd)
        torch.cuda.synchronize()
        assert torch.isfinite(torch.view_as_real(V)).all()
        if ref is None:
            ref = V.clone()
        else:
            assert torch.equal(V, ref), f"tile {tile} differs from the default at M = {M}"


def test_tiles_that_do_not_fit_are_rejected(device):
    from paper_2501_05244_amd.api import plan_from_workload
    w, _ = case(seed=3, L=200, F=4)
    for M, tile in ((1024, 1601), (1024, 116), (128, 303)):
        print(f"case: reject M {M} tile {tile}", flush=True)
        with pytest.raises(RuntimeError):
            plan_from_workload(w, device, M=M, spread_tile=tile)
