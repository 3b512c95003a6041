"""Writes method_gap.txt: how far NURSD is from the physical RSD sum.

NURSD evaluates the RSD convolution on a frame of pitch dx/q (the NUFFT
section: relay samples enter through a type-1 NUFFT, the kernel is sampled
on the frame), while eq. PF_RSD_Defn sums the kernel at every relay sample
directly.  The paper calls the difference negligible for well-sampled relays;
this script reports it per workload and per upsampling q as the rel-L2 gap
between the oracle's NURSD operator (O1: nursd_grid, srsd, nursd_points,
srsd_points) and the brute-force sum (O2: rsd_direct), on the workloads' own
phasors (rendered scenes) restricted to a seeded subset of bins, planes and
voxels.  It calls only oracle/ and the input generators.

    python tests/golden/method_gap.py            (about 5 minutes on 8 cores)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import nursd_ref as o  # noqa: E402
from workloads import scenes  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "method_gap.txt")
VOX_PER_PLANE = 1024


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def pick(n, k):
    """k evenly spaced indices of range(n)."""
    return np.unique(np.round(np.linspace(0, n - 1, k)).astype(int))


def grid_case(w, P, f, bsel, zsel, qs, rng):
    g = w.grid
    sub = scenes.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny, np.asarray(g.z)[zsel])
    vox = o.grid_voxels(sub)                                  # [Z*ny*nx][3]
    per = g.nx * g.ny
    take = np.concatenate([iz * per + np.sort(rng.choice(per, min(VOX_PER_PLANE, per), replace=False))
                           for iz in range(len(zsel))])
    ref = o.rsd_direct(P[bsel], w.relay_xy.astype(np.float64), f[bsel], vox[take], w.xp, chunk=256)
    rows = []
    for q in qs:
        fr = o.frame_for_workload(w, q)
        V = o.nursd_grid(P[bsel], w.relay_xy.astype(np.float64), f[bsel], fr, sub, w.xp).reshape(-1)[take]
        rows.append((q, fr.M, rel(V, ref), rel(np.abs(V), np.abs(ref)), len(take)))
    return rows


def srsd_case(w, P, f, bsel, zsel, rng):
    g = w.grid
    N = g.nx
    z = np.asarray(g.z)[zsel]
    alphas = o.srsd_alpha(z, w.zref)
    fr = o.frame_for_workload(w, 1)
    sub = scenes.Grid(g.x0, g.y0, g.dx, g.dy, N, N, z)
    V = o.srsd(P[bsel], w.relay_xy.astype(np.float64), f[bsel], fr, sub, w.xp, alphas)    # [Z][N][N]
    m = np.arange(N) - N // 2
    vox, vals = [], []
    for iz in range(len(z)):
        pick_ = np.sort(rng.choice(N * N, VOX_PER_PLANE, replace=False))
        iy, ix = pick_ // N, pick_ % N
        x = fr.cx + m[ix] * fr.dx / alphas[iz]
        y = fr.cy + m[iy] * fr.dy / alphas[iz]
        vox.append(np.stack([x, y, np.full(len(x), z[iz])], axis=1))
        vals.append(V[iz].reshape(-1)[pick_])
    ref = o.rsd_direct(P[bsel], w.relay_xy.astype(np.float64), f[bsel], np.concatenate(vox), w.xp, chunk=256)
    Vs = np.concatenate(vals)
    return [(1, fr.M, rel(Vs, ref), rel(np.abs(Vs), np.abs(ref)), len(Vs))]


def points_case(w, P, f, bsel, zsel, rng, scaled):
    z = np.asarray(w.grid.z)[zsel]
    ptr = w.plane_ptr
    xy, sptr = [], [0]
    for iz in zsel:
        a, e = int(ptr[iz]), int(ptr[iz + 1])
        k = np.sort(rng.choice(e - a, min(VOX_PER_PLANE, e - a), replace=False))
        xy.append(w.voxel_xy[a:e][k].astype(np.float64))
        sptr.append(sptr[-1] + len(k))
    vxy = np.concatenate(xy)
    sptr = np.asarray(sptr)
    fr = o.frame_for_workload(w, 1)
    relay = w.relay_xy.astype(np.float64)
    if scaled:
        V = o.srsd_points(P[bsel], relay, f[bsel], fr, w.grid.nx, z, o.srsd_alpha(z, w.zref), sptr, vxy, w.xp)
    else:
        V = o.nursd_points(P[bsel], relay, f[bsel], fr, z, sptr, vxy, w.xp)
    vz = np.repeat(z, np.diff(sptr))
    ref = o.rsd_direct(P[bsel], relay, f[bsel], np.column_stack([vxy, vz]), w.xp, chunk=256)
    return [(1, fr.M, rel(V, ref), rel(np.abs(V), np.abs(ref)), len(V))]


def tiny_rows():
    """The tiny workload (31.25 mm pitch, above half the shortest
    wavelength): all 16 bins, 4 planes, every voxel; q = 1, 2, 4."""
    w = scenes.config_tiny(render=True)
    P, f = o.phasors_from_workload(w)
    rng = np.random.default_rng(71)
    return grid_case(w, P, f, np.arange(len(f)), pick(len(w.grid.z), 4), (1, 2, 4), rng)


def main():
    lines = ["# workload | q | M | bins | planes | voxels | gap complex V | gap |V|"]

    def emit(name, rows, nb, nz):
        for q, M, gv, gi, nv in rows:
            lines.append(f"{name} | {q} | {M} | {nb} | {nz} | {nv} | {gv:.4e} | {gi:.4e}")
            print(lines[-1], flush=True)

    t = time.time()
    emit("tiny", tiny_rows(), 16, 4)
    spad = scenes.config_spad(render=True)
    P, f = o.phasors_from_workload(spad)
    bsel = pick(len(f), 4)
    rng = np.random.default_rng(72)
    emit("spad", grid_case(spad, P, f, bsel, pick(len(spad.grid.z), 4), (1, 2), rng), 4, 4)
    w = scenes.config_srsd(render=False)
    emit("srsd", srsd_case(w, P, f, bsel, pick(len(w.grid.z), 4), np.random.default_rng(73)), 4, 4)
    w = scenes.config_frustum_points(render=False)
    emit("frustum_points", points_case(w, P, f, bsel, pick(len(w.grid.z), 4), np.random.default_rng(74), False),
         4, 4)
    w = scenes.config_srsd_points(render=False)
    emit("srsd_points", points_case(w, P, f, bsel, pick(len(w.grid.z), 4), np.random.default_rng(75), True), 4, 4)
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {OUT} in {time.time() - t:.0f} s")


if __name__ == "__main__":
    main()
