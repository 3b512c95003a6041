"""Benchmark: NURSD reconstruction throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: the SPAD-scale reconstruction (65,536 relay samples from a 32x32
SPAD array at 64 oblique poses over 2x2 m, 4,096 bins at 4 ps, 200 points
and two patches, 6 cm wavelength with 96 frequencies, 256x256x128 voxels,
FFT size 512).  One step is one full forward from histograms already
resident in HBM: temporal phasor transform, type-1 NUFFT, per-depth RSD
propagation of every (frequency, plane) pair, coherent volume and
intensity.  The metric is voxel-frequency propagations per second
(256*256*128*96 per step).

Prints one JSON line.  The timed steps run without instrumentation; the
roofline object describes the dominant kernel, whose launches are timed with
HIP events on their stream during as many further steps run right after the
timed ones.  cpu_baseline times the FP64 oracle on a bounded sample of the
same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Non-packed FP32 vector issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x
# 2 FLOP per FMA x 2.4 GHz (packed FP32 instructions are not used).
PEAK_FP32_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0


def fft_flops(n: int) -> float:
    return 5.0 * n * math.log2(n)


def stage_work(stage: str, info: dict, w) -> tuple[float, float]:
    """Algorithmic work of one forward for a stage: (flops, bytes).

    Flops count 5 n log2 n per n-point complex FFT and 6 per complex multiply.
    Bytes are the HBM traffic the stage's data flow needs at minimum: each
    intermediate written once and read once, the spectrum U of a frequency read
    once per launch; for the propagation passes (per (frequency, depth) plane,
    H = M/2): kernel_rows writes the (H+1)^2 quadrant spectrum, propagate_cols
    reads it and writes M x ny column transforms, propagate_rows reads those and
    read-modify-writes the ny x nx plane once per frequency chunk."""
    M, Mf, F, L = info["M"], info["Mf"], info["n_freq"], info["n_relay"]
    g = w.grid
    Z, nx, ny = len(g.z), g.nx, g.ny
    planes = F * Z
    H = M // 2
    fc = info.get("freq_chunk", 8)
    if stage == "propagate_cols":
        launches = planes / (fc * info.get("plane_chunk", 16))
        return (planes * ((H + 1 + M) * fft_flops(M) + 6.0 * M * M),
                planes * (8.0 * (H + 1) ** 2 + 8.0 * M * ny) + launches * fc * 8.0 * M * M)
    if stage == "propagate_rows":
        return (planes * (ny * fft_flops(M) + 8.0 * nx * ny),
                planes * 8.0 * M * ny + (planes / fc) * 16.0 * nx * ny)
    if stage == "kernel_rows":
        return planes * (H + 1) * fft_flops(M), planes * 8.0 * (H + 1) ** 2
    if stage == "spread":
        return F * L * 49 * 8.0 + F * (Mf // 2) * fft_flops(Mf), F * (L * 12.0 + 8.0 * Mf * Mf)
    if stage == "phasor":
        return 8.0 * L * w.wavelet.n_time * F, float(L * w.wavelet.n_time * 4 + F * L * 8)
    if stage == "fine_y":
        return F * M * fft_flops(Mf), float(F * M * Mf * 8 + F * M * M * 8)
    return 0.0, 0.0


def path_model_bytes(info: dict, w) -> float:
    """Streaming model of the whole forward: per (frequency, depth) plane
    24 M^2 + 16 M N + 16 N^2 bytes (generate kernel and column FFT; row FFT,
    spectrum multiply and row inverse; column inverse, crop and accumulate),
    plus one read of the histogram.  The type-1 steps are left out, which
    makes the fraction conservative."""
    M, F = info["M"], info["n_freq"]
    g = w.grid
    N = max(g.nx, g.ny)
    return F * len(g.z) * (24.0 * M * M + 16.0 * M * N + 16.0 * N * N) + w.relay_xy.shape[0] * w.wavelet.n_time * 4.0


def host_cpu() -> dict:
    """CPU model, logical CPUs visible to this process, and the threads
    numpy's BLAS (the oracle's matrix products) runs with."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        visible = len(os.sched_getaffinity(0))
    except AttributeError:
        visible = os.cpu_count() or 1
    blas = None
    try:
        from threadpoolctl import threadpool_info
        blas = max((p["num_threads"] for p in threadpool_info() if p.get("user_api") == "blas"), default=None)
    except Exception:
        blas = None
    return {"model": model, "nproc": visible, "blas_threads": blas}


def cpu_baseline(w, hist, reps: int = 3) -> dict:
    """Oracle (FP64, numpy) on 4 of the 96 frequencies and 8 of the 128 planes,
    full 256x256 lateral window, phasor transform included; median of `reps`
    runs."""
    from oracle import nursd_ref as o
    from workloads import scenes
    wl = w.wavelet
    bins, f = o.wavelet_bins(wl.lambda_c, wl.n_time, wl.dt, wl.n_freq)
    sel_b = np.array([10, 34, 58, 82])
    sel_z = np.arange(0, 128, 16)[:8]
    g = w.grid
    sub = scenes.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny, g.z[sel_z])
    fr = o.frame_for_workload(w)
    times = []
    for _ in range(reps):
        t = time.perf_counter()
        wts = o.phasor_weights(f[sel_b], wl.lambda_c, wl.sigma_rel, wl.t0)
        P = o.temporal_phasor(hist, bins[sel_b], wts)
        o.nursd_grid(P, w.relay_xy.astype(np.float64), f[sel_b], fr, sub, w.xp)
        times.append(time.perf_counter() - t)
    dt = float(np.median(times))
    units = g.nx * g.ny * len(sel_z) * len(sel_b)
    cpu = host_cpu()
    return {"value": units / dt, "unit": "voxel*freq/s", "cores": cpu["blas_threads"] or cpu["nproc"],
            "kind": "oracle", "cpu_model": cpu["model"], "nproc": cpu["nproc"],
            "sample": f"{len(sel_b)} of 96 frequencies x {len(sel_z)} of 128 planes, full 256x256 window; "
                      f"phasor DFT + direct NUDFT-1 + direct 2D DFTs in float64; median of {reps} runs "
                      f"({', '.join(f'{x:.2f}' for x in times)} s)"}


def time_ms(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def secondary(w_spad, dev) -> dict:
    """The other hot-path rows on their own workloads: scaled RSD frustum,
    NURSD-3 voxel lists, scaled RSD at voxel lists, 3D NURSD, 4D video, several
    illumination positions, the compression gather, forward + adjoint, and
    batched vs plain serving."""
    import torch
    from paper_2501_05244_amd.api import Batch, plan_from_workload
    from paper_2501_05244_amd.autograd import nursd
    from workloads import scenes
    out = {}
    hist = torch.from_numpy(w_spad.hist).to(dev)
    # scaled RSD: 256x256 samples on 128 planes over [1,4] m, 96 frequencies
    w = scenes.config_srsd(render=False)
    plan = plan_from_workload(w, dev)
    I = torch.empty(plan.out_shape(), dtype=torch.float32, device=dev)
    ms = time_ms(lambda: plan.forward_hist(hist, vol=False, out_I=I), 5)
    out["srsd"] = {"workload": "srsd_L65536_F96_256x256x128_frustum_1-4m", "ms": round(ms, 3),
                   "voxel*freq/s": scenes.work_units(w) / (ms * 1e-3)}
    del plan
    # NURSD-3: 1,048,576 jittered frustum voxels on 64 planes, 96 frequencies
    w = scenes.config_frustum_points(render=False)
    plan = plan_from_workload(w, dev)
    I = torch.empty(plan.out_shape(), dtype=torch.float32, device=dev)
    ms = time_ms(lambda: plan.forward_hist(hist, vol=False, out_I=I), 3)
    out["nursd3_points"] = {"workload": "points_L65536_F96_1048576vox_64planes", "ms": round(ms, 3),
                            "voxel*freq/s": scenes.work_units(w) / (ms * 1e-3)}
    del plan
    # scaled RSD at voxel lists: the same 1,048,576 frustum voxels on 64 scaled planes
    w = scenes.config_srsd_points(render=False)
    plan = plan_from_workload(w, dev)
    I = torch.empty(plan.out_shape(), dtype=torch.float32, device=dev)
    ms = time_ms(lambda: plan.forward_hist(hist, vol=False, out_I=I), 3)
    out["srsd_points"] = {"workload": "srsd_points_L65536_F96_1048576vox_64planes", "ms": round(ms, 3),
                          "voxel*freq/s": scenes.work_units(w) / (ms * 1e-3)}
    del plan
    # 3D NURSD: the SPAD samples on a curved wall (depth within +-5 cm)
    w = scenes.config_nonplanar()
    plan = plan_from_workload(w, dev)
    P3 = plan.phasor(hist)
    I = torch.empty(plan.out_shape(), dtype=torch.float32, device=dev)
    ms = time_ms(lambda: plan.forward_phasor(P3, vol=False, out_I=I), 3)
    out["nursd3d"] = {"workload": "nonplanar_L65536_F96_256x256x128_depthgrid%d" % plan.info["depth3d"], "ms": round(ms, 3),
                      "voxel*freq/s": scenes.work_units(w) / (ms * 1e-3)}
    del plan, P3
    # 4D light transport: 32 frames at 50 ps of the SPAD volume
    w = scenes.config_spad(render=False)
    plan = plan_from_workload(w, dev)
    P = plan.phasor(hist)
    T = 32
    ms = time_ms(lambda: plan.forward_video(P, T, -0.8e-9, 0.05e-9, vol=False), 3)
    out["video"] = {"workload": "spad_L65536_F96_256x256x128_32frames", "ms": round(ms, 3),
                    "voxel*freq/s": scenes.work_units(w) / (ms * 1e-3),
                    "voxel*frame/s": w.grid.nx * w.grid.ny * len(w.grid.z) * T / (ms * 1e-3)}
    # four illumination positions sharing every kernel spectrum
    K = 4
    Pk = P.unsqueeze(0).expand(K, -1, -1).contiguous()
    xps = [[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0.0, 0.5, 0.0], [-0.5, -0.5, 0.0]]
    ms = time_ms(lambda: plan.forward_multi(Pk, xps, vol=False), 3)
    out["multi_illumination"] = {"workload": "spad_L65536_F96_256x256x128_4positions", "ms": round(ms, 3),
                                 "voxel*freq*position/s": K * scenes.work_units(w) / (ms * 1e-3)}
    # compression preprocessing: stride-2 lattice fill of 96 x 256 x 256 grid phasors
    from paper_2501_05244_amd.api import subsample_nearest
    Pg = P[:, :65536].reshape(96, 256, 256).contiguous()
    ms = time_ms(lambda: subsample_nearest(Pg, 2), 10)
    out["subsample_nearest"] = {"workload": "F96_256x256_stride2", "ms": round(ms, 4),
                                "GB/s": 2 * Pg.numel() * 8 / (ms * 1e-3) / 1e9}
    del plan, P, Pk, Pg
    # differentiation: forward + adjoint (grad P and grad xy) through autograd
    w = scenes.config_diff()
    plan = plan_from_workload(w, dev)
    P = plan.phasor(torch.from_numpy(w.hist).to(dev))
    xy = torch.from_numpy(w.relay_xy).to(dev)
    tgt = torch.zeros(plan.out_shape(), dtype=torch.complex64, device=dev)

    V = torch.empty(plan.out_shape(), dtype=torch.complex64, device=dev)
    ms = time_ms(lambda: plan.forward_phasor(P, out_vol=V, intensity=False), 10)
    out["diff_forward"] = {"workload": "diff_L16384_F48_128x128x64", "ms": round(ms, 3),
                           "voxel*freq/s": scenes.work_units(w) / (ms * 1e-3)}

    def step():
        Pg = P.detach().requires_grad_(True)
        xg = xy.detach().requires_grad_(True)
        loss = (nursd(Pg, xg, plan) - tgt).abs().pow(2).sum()
        loss.backward()
    ms = time_ms(step, 5)
    out["forward_adjoint"] = {"workload": "diff_L16384_F48_128x128x64", "ms": round(ms, 3),
                              "voxel*freq/s (forward+adjoint)": scenes.work_units(w) / (ms * 1e-3)}
    del plan
    # batched serving of 64 uneven scenes vs the plain per-scene loop
    ws = scenes.config_batch()
    plans = [plan_from_workload(x, dev) for x in ws]
    hists = [torch.from_numpy(x.hist).to(dev) for x in ws]
    outs = [torch.empty(p.out_shape(), dtype=torch.float32, device=dev) for p in plans]
    units = sum(scenes.work_units(x) for x in ws)

    def plain():
        for p, h, o in zip(plans, hists, outs):
            p.forward_hist(h, vol=False, out_I=o)
    t_plain = time_ms(plain, 3)
    ref = [o.clone() for o in outs]
    b = Batch(plans, autotune=True)
    bouts = [torch.empty_like(o) for o in outs]
    b.forward(hists, bouts)
    t_batch = time_ms(lambda: b.forward(hists, bouts), 5)
    err = max(float((x - y).norm() / y.norm()) for x, y in zip(bouts, ref))
    info = b.info()
    out["batched"] = {"workload": "64 scenes: relays 2k-64k, grids 64^2x32..256^2x128, F 16-128, 4-8 cm",
                      "plain_ms": round(t_plain, 3), "batched_ms": round(t_batch, 3),
                      "speedup": round(t_plain / t_batch, 4), "max_rel_l2_batched_vs_plain": err,
                      "voxel*freq/s": units / (t_batch * 1e-3),
                      "autotuned": {k: info[k] for k in ("rounds", "schedule", "serial", "shared_kernels", "kernel_choices")},
                      "workspace_bytes": info["workspace_bytes"]}
    return out


KERNEL_SOURCES = ("k_rsd.hip", "k_nufft.hip", "k_phasor.hip", "kernels.hpp", "wavefft.hpp", "fft.hpp", "persistent.hpp",
                  "api.hip", "host_plan.hpp")


def kernel_source_hash() -> str:
    """SHA-256 over the sources of the forward kernels and of the host code
    that chunks their launches and bins the relay samples; a counter summary
    taken on other sources no longer describes the launches that run."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2501_05244_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def load_counters(name: str):
    """A committed rocprofv3 counter summary (profiles/<name>.json), if it
    exists and was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"{name}.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return d


def load_traffic(stage: str):
    """HBM bytes per launch of `stage` (FETCH_SIZE and WRITE_SIZE, scaled by
    the copy calibration), or None."""
    d = load_counters(f"{stage}_spad_counters")
    return None if d is None else d.get("hbm_bytes_per_launch")


def copy_calibration(dev) -> None:
    """A plain device-to-device copy of 256 MiB, five times: the reference
    whose FETCH_SIZE / WRITE_SIZE readings scale the counters of the hot
    kernels to bytes (each dispatch reads and writes exactly 256 MiB)."""
    import torch
    n = 256 << 20
    src = torch.ones(n // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_dispatch": n, "dispatches": 5}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the plain copy used to scale rocprofv3 byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the reconstruction would shard "
              "by depth plane with no exchange); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2501_05244_amd.api import plan_from_workload
    from workloads import scenes

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        copy_calibration(dev)
        return
    w = scenes.config_spad()
    plan = plan_from_workload(w, dev)
    hist = torch.from_numpy(w.hist).to(dev)
    g = w.grid
    shape = (len(g.z), g.ny, g.nx)
    V = torch.empty(shape, dtype=torch.complex64, device=dev)
    I = torch.empty(shape, dtype=torch.float32, device=dev)
    units = g.nx * g.ny * len(g.z) * plan.F

    for _ in range(args.warmup):
        plan.forward_hist(hist, out_vol=V, out_I=I)
    # untimed profiled pass: find the dominant kernel
    torch.cuda.synchronize()
    plan.profile_begin()
    plan.forward_hist(hist, out_vol=V, out_I=I)
    stages = plan.profile_end()
    dominant = max(stages, key=lambda k: stages[k][0])

    # The K timed steps run without instrumentation (per-launch events cost
    # about 0.3 ms per forward at this workload).
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        plan.forward_hist(hist, out_vol=V, out_I=I)
    e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = e0.elapsed_time(e1) / args.steps
    wall_ms = (t1 - t0) * 1e3 / args.steps
    # Then K more steps with HIP events recorded on the launch stream around
    # every launch of the dominant kernel: its average launch duration.
    plan.profile_begin([dominant])
    for _ in range(args.steps):
        plan.forward_hist(hist, out_vol=V, out_I=I)
    torch.cuda.synchronize()
    dom = plan.profile_end()[dominant]

    flops, nbytes = stage_work(dominant, plan.info, w)
    launches_per_step = dom[1] / args.steps
    avg_launch_ms = dom[0] / dom[1]
    sec_per_launch = avg_launch_ms * 1e-3
    alu = {"bound": "alu", "achieved": round(flops / launches_per_step / sec_per_launch / 1e12, 2),
           "peak": round(PEAK_FP32_TFLOPS, 2), "unit": "TFLOP/s"}
    alu["frac"] = round(alu["achieved"] / alu["peak"], 4)
    hbm = {"bound": "hbm", "achieved": round(nbytes / launches_per_step / sec_per_launch / 1e9, 1),
           "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    hbm["frac"] = round(hbm["achieved"] / hbm["peak"], 4)
    roof, other = (alu, hbm) if alu["frac"] >= hbm["frac"] else (hbm, alu)
    roof["traffic"] = load_traffic(dominant)
    roof["kernel"] = dominant
    roof["avg_launch_ms"] = round(avg_launch_ms, 4)
    roof["launch_timing"] = (f"HIP events on the launch stream around each of the {dom[1]} launches of "
                             f"{args.steps} further steps run right after the timed ones")
    roof["algorithmic_per_launch"] = {"flop": flops / launches_per_step, "bytes": nbytes / launches_per_step}
    roof["other_bound"] = other
    # Whole-forward HBM traffic measured by rocprofv3 (sum over every
    # dispatch of one forward), from the committed counter summary.
    fwd = load_counters("spad_forward_hbm")
    measured = None
    if fwd is not None:
        b = float(fwd["hbm_bytes_per_forward"])
        measured = {"bytes_per_step": b, "GBs": round(b / (ms * 1e-3) / 1e9, 1),
                    "frac_of_peak": round(b / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                    "source": "profiles/spad_forward_hbm_counters.md"}
    # A streaming model of the propagation (a figure of the model, not of the
    # bytes this design moves: it counts a full M^2 kernel spectrum per plane
    # where only the quadrant is stored).
    model = {"bytes_per_step": path_model_bytes(plan.info, w),
             "note": "streaming-model bytes (24M^2+16MN+16N^2 per plane + histogram); not measured traffic"}

    out = {
        "metric": "NURSD voxel*freq propagations/s at rel-L2<=1e-4; batched vs plain speedup",
        "value": units / (ms * 1e-3),
        "unit": "voxel*freq/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "wall_ms_per_step": round(wall_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "spad_L65536_T4096_F96_256x256x128_M512", "relay_samples": w.relay_xy.shape[0],
                   "time_bins": w.wavelet.n_time, "frequencies": plan.F, "voxels": [g.nx, g.ny, len(g.z)],
                   "fft_size": plan.M, "complex": "c64 data, f64 phase arguments"},
        "stage_ms_per_step": {k: round(v[0], 4) for k, v in stages.items()},
        "roofline": roof,
        "measured_hbm_whole_forward": measured,
        "streaming_model": model,
    }
    if not args.no_secondary:
        del V, I
        torch.cuda.empty_cache()
        sec = secondary(w, dev)
        out["batched_vs_plain_speedup"] = sec["batched"]["speedup"]
        out["secondary"] = sec
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, w.hist)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
