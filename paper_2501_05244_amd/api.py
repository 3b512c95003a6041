"""PyTorch-facing wrapper around the C ABI: device memory and streams only.

Every step of the reconstruction runs in the HIP kernels of libnursd.so;
this module allocates output tensors and the workspace with torch, passes
raw device pointers and the current HIP stream, and raises on any error.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, byref, c_double, c_int32, c_size_t, c_void_p

import numpy as np
import torch

from . import _lib
from ._lib import (MODE_GRID, MODE_GRID3D, MODE_POINTS, MODE_SRSD, MODE_SRSD_POINTS, Geometry, Options, PlanInfo,
                   Wavelet, check)


def _stream(stream=None) -> c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return c_void_p(s.cuda_stream)


def _ptr(t) -> c_void_p:
    return c_void_p(0 if t is None else t.data_ptr())


def _need(t: torch.Tensor, dtype, shape, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Plan:
    """One reconstruction geometry (C handle nursd_plan)."""

    def __init__(self, relay_xy: torch.Tensor, *, lambda_c: float, n_time: int, dt: float, t0: float,
                 n_freq: int, z, mode: int = MODE_GRID, x0=0.0, y0=0.0, dx=1.0, dy=1.0, nx=0, ny=0,
                 bins=None, coherent=True, sigma_rel=0.2, pad=2.0, tol=1e-6, M=0, freq_chunk=0,
                 plane_chunk=0, xp=(0.0, 0.0, 0.0), zref=0.0, alpha=None, plane_ptr=None,
                 voxel_xy: torch.Tensor | None = None, relay_z: torch.Tensor | None = None, z_mid=0.0, dz3=0.0,
                 mz3=0, kernel_inv_r=True, upsample_q=1, weights: torch.Tensor | None = None, spread_tile=0,
                 stream=None):
        self._lib = _lib.load()
        self.handle = None
        L = relay_xy.shape[0]
        _need(relay_xy, torch.float32, (L, 2), "relay_xy")
        self.L = L
        self.mode = mode
        self.coherent = bool(coherent)
        wl = Wavelet()
        geo = Geometry()
        opt = Options()
        self._lib.nursd_default_options(byref(wl), byref(geo), byref(opt))
        wl.lambda_c, wl.n_time, wl.dt, wl.t0, wl.n_freq = lambda_c, n_time, dt, t0, n_freq
        wl.sigma_rel = sigma_rel
        wl.coherent = 1 if coherent else 0
        wl.kernel_inv_r = 1 if kernel_inv_r else 0
        self._keep = []
        if bins is not None:
            b = np.ascontiguousarray(bins, dtype=np.int32)
            self._keep.append(b)
            wl.bins = b.ctypes.data_as(POINTER(c_int32))
            wl.n_freq = len(b)
        zz = np.ascontiguousarray(z, dtype=np.float64)
        self._keep.append(zz)
        geo.mode = mode
        geo.x0, geo.y0, geo.dx, geo.dy, geo.nx, geo.ny = x0, y0, dx, dy, nx, ny
        geo.nz = len(zz)
        geo.z = zz.ctypes.data_as(POINTER(c_double))
        geo.zref = zref
        for i in range(3):
            geo.xp[i] = float(xp[i])
        if alpha is not None:
            al = np.ascontiguousarray(alpha, dtype=np.float64)
            self._keep.append(al)
            geo.alpha = al.ctypes.data_as(POINTER(c_double))
        if plane_ptr is not None:
            pp = np.ascontiguousarray(plane_ptr, dtype=np.int32)
            self._keep.append(pp)
            geo.plane_ptr = pp.ctypes.data_as(POINTER(c_int32))
        if voxel_xy is not None:
            _need(voxel_xy, torch.float32, (voxel_xy.shape[0], 2), "voxel_xy")
            self.voxel_xy = voxel_xy
            geo.voxel_xy_dev = voxel_xy.data_ptr()
        if relay_z is not None:
            _need(relay_z, torch.float32, (L,), "relay_z")
            self.relay_z = relay_z
            geo.relay_z_dev = relay_z.data_ptr()
        geo.z_mid, geo.dz3, geo.mz3 = z_mid, dz3, mz3
        opt.n_relay = L
        opt.pad, opt.tol, opt.M = pad, tol, M
        opt.freq_chunk, opt.plane_chunk = freq_chunk, plane_chunk
        opt.upsample_q = int(upsample_q)
        opt.spread_tile = int(spread_tile)
        if weights is not None:
            _need(weights, torch.float32, (L,), "weights")
            opt.weights_dev = weights.data_ptr()      # copied by nursd_plan_create
        h = c_void_p()
        check(self._lib.nursd_plan_create(byref(wl), byref(geo), byref(opt), _ptr(relay_xy), _stream(stream),
                                          byref(h)), "nursd_plan_create")
        self.handle = h
        info = PlanInfo()
        check(self._lib.nursd_plan_info(self.handle, byref(info)), "nursd_plan_info")
        self.info = {k: getattr(info, k) for k, _ in PlanInfo._fields_}
        self.F = self.info["n_freq"]
        self.M = self.info["M"]
        self.nx, self.ny, self.nz = nx, ny, len(zz)
        self.n_time = n_time
        self.device = relay_xy.device
        self._ws = None

    def __del__(self):
        if getattr(self, "handle", None):
            self._lib.nursd_plan_destroy(self.handle)
            self.handle = None

    # ------------------------------------------------------------ workspace
    def workspace(self) -> tuple[torch.Tensor, int]:
        n = int(self.info["workspace_bytes"])
        if self._ws is None or self._ws.numel() < n + 256:
            self._ws = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        off = (-base) % 256
        return self._ws, base + off

    def _ws_args(self):
        _, p = self.workspace()
        return c_void_p(p), c_size_t(int(self.info["workspace_bytes"]))

    def out_shape(self):
        if self.mode in (MODE_POINTS, MODE_SRSD_POINTS):
            return (self.info["n_voxels"],)
        return (self.nz, self.ny, self.nx)

    # ------------------------------------------------------------ profiling
    def profile_begin(self, stages=None):
        mask = 0xFFFFFFFF if stages is None else sum(1 << _lib.STAGES.index(n) for n in stages)
        check(self._lib.nursd_profile_begin(self.handle, mask), "nursd_profile_begin")

    def profile_end(self) -> dict:
        ms = (c_double * _lib.NUM_STAGES)()
        calls = (c_int32 * _lib.NUM_STAGES)()
        check(self._lib.nursd_profile_end(self.handle, ms, calls), "nursd_profile_end")
        return {n: (ms[i], calls[i]) for i, n in enumerate(_lib.STAGES) if calls[i]}

    # ------------------------------------------------------------ entry points
    def set_points(self, relay_xy: torch.Tensor, stream=None):
        _need(relay_xy, torch.float32, (self.L, 2), "relay_xy")
        # whatever tensor autograd bound before no longer describes the plan
        self._bound_xy = None
        check(self._lib.nursd_plan_set_points(self.handle, _ptr(relay_xy), _stream(stream)),
              "nursd_plan_set_points")

    def bind_points(self, relay_xy: torch.Tensor, stream=None):
        """Make the plan use the positions held in `relay_xy` (a [L][2]
        float tensor), re-binning only when the plan does not already hold
        exactly that memory at its current version (autograd calls this for
        every forward and backward).  The plan keeps a reference to the
        bound memory, so its address cannot be freed and reused by another
        tensor while it is bound; tensors that share it (detach(), views of
        the same contiguous layout) share its version counter, so an
        in-place change to them is seen too."""
        bound = getattr(self, "_bound_xy", None)
        if (bound is not None and relay_xy.is_contiguous() and relay_xy.data_ptr() == bound[0].data_ptr()
                and relay_xy._version == bound[1]):
            return
        src = relay_xy.detach().contiguous()
        self.set_points(src, stream)
        self._bound_xy = (src, relay_xy._version)

    def phasor(self, hist: torch.Tensor, stream=None) -> torch.Tensor:
        _need(hist, torch.float32, (self.L, self.n_time), "hist")
        P = torch.empty((self.F, self.L), dtype=torch.complex64, device=self.device)
        check(self._lib.nursd_phasor(self.handle, _ptr(hist), _ptr(P), _stream(stream)), "nursd_phasor")
        return P

    def spectrum(self, P: torch.Tensor, stream=None) -> torch.Tensor:
        _need(P, torch.complex64, (self.F, self.L), "P")
        U = torch.empty((self.F, self.M, self.M), dtype=torch.complex64, device=self.device)
        ws, n = self._ws_args()
        check(self._lib.nursd_spectrum(self.handle, _ptr(P), _ptr(U), ws, n, _stream(stream)), "nursd_spectrum")
        return U

    def _outs(self, vol, intensity, out_vol=None, out_I=None):
        V = I = None
        if vol and self.coherent:
            V = out_vol if out_vol is not None else torch.empty(self.out_shape(), dtype=torch.complex64,
                                                                 device=self.device)
        if intensity:
            I = out_I if out_I is not None else torch.empty(self.out_shape(), dtype=torch.float32,
                                                            device=self.device)
        return V, I

    def forward_hist(self, hist: torch.Tensor, vol=True, intensity=True, out_vol=None, out_I=None,
                     stream=None):
        _need(hist, torch.float32, (self.L, self.n_time), "hist")
        V, I = self._outs(vol, intensity, out_vol, out_I)
        ws, n = self._ws_args()
        check(self._lib.nursd_forward_hist(self.handle, _ptr(hist), _ptr(V), _ptr(I), ws, n, _stream(stream)),
              "nursd_forward_hist")
        return V, I

    def forward_hist_static(self, hist: torch.Tensor, out_vol=None, out_I=None, stream=None):
        """nursd_forward_hist on the library's fixed device scratch: the call
        itself allocates nothing (pass out_vol / out_I to keep it so)."""
        _need(hist, torch.float32, (self.L, self.n_time), "hist")
        V, I = self._outs(out_vol is not None or out_I is None, True, out_vol, out_I) \
            if out_vol is None and out_I is None else (out_vol, out_I)
        check(self._lib.nursd_forward_hist_static(self.handle, _ptr(hist), _ptr(V), _ptr(I), _stream(stream)),
              "nursd_forward_hist_static")
        return V, I

    def forward_phasor(self, P: torch.Tensor, vol=True, intensity=True, out_vol=None, out_I=None,
                       stream=None):
        _need(P, torch.complex64, (self.F, self.L), "P")
        V, I = self._outs(vol, intensity, out_vol, out_I)
        ws, n = self._ws_args()
        check(self._lib.nursd_forward_phasor(self.handle, _ptr(P), _ptr(V), _ptr(I), ws, n, _stream(stream)),
              "nursd_forward_phasor")
        return V, I

    def forward_video(self, P: torch.Tensor, n_frames: int, t_first: float, t_step: float, vol=True,
                      intensity=True, stream=None):
        """4D light transport: frames [n_frames][nz][ny][nx] of the coherent
        field (complex) and/or its magnitude at t_first + j t_step."""
        _need(P, torch.complex64, (self.F, self.L), "P")
        shape = (n_frames,) + self.out_shape()
        V = torch.empty(shape, dtype=torch.complex64, device=self.device) if vol else None
        I = torch.empty(shape, dtype=torch.float32, device=self.device) if intensity else None
        n = c_size_t()
        check(self._lib.nursd_video_workspace_size(self.handle, byref(n)), "nursd_video_workspace_size")
        if getattr(self, "_vws", None) is None or self._vws.numel() < n.value + 256:
            self._vws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        base = self._vws.data_ptr()
        ws = c_void_p(base + (-base) % 256)
        check(self._lib.nursd_forward_video(self.handle, _ptr(P), n_frames, float(t_first), float(t_step), _ptr(V),
                                            _ptr(I), ws, n, _stream(stream)), "nursd_forward_video")
        return V, I

    def forward_multi(self, P: torch.Tensor, xps, vol=True, intensity=True, stream=None):
        """Several illumination positions: P [K][F][L] phasors measured under
        each position, xps [K][3]; returns the summed volume and/or |V|."""
        K = P.shape[0]
        _need(P, torch.complex64, (K, self.F, self.L), "P")
        xp = np.ascontiguousarray(np.asarray(xps, dtype=np.float64).reshape(K, 3))
        V, I = self._outs(vol, intensity)
        n = c_size_t()
        check(self._lib.nursd_multi_workspace_size(self.handle, K, byref(n)), "nursd_multi_workspace_size")
        if getattr(self, "_mws", None) is None or self._mws.numel() < n.value + 256:
            self._mws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        base = self._mws.data_ptr()
        ws = c_void_p(base + (-base) % 256)
        check(self._lib.nursd_forward_multi(self.handle, _ptr(P), K, xp.ctypes.data_as(POINTER(c_double)), _ptr(V),
                                            _ptr(I), ws, n, _stream(stream)), "nursd_forward_multi")
        return V, I

    def adjoint(self, grad_vol: torch.Tensor, P: torch.Tensor | None = None, stream=None):
        _need(grad_vol, torch.complex64, self.out_shape(), "grad_vol")
        gP = torch.empty((self.F, self.L), dtype=torch.complex64, device=self.device)
        gxy = None
        if P is not None:
            _need(P, torch.complex64, (self.F, self.L), "P")
            gxy = torch.empty((self.L, 2), dtype=torch.float32, device=self.device)
        ws, n = self._ws_args()
        check(self._lib.nursd_adjoint(self.handle, _ptr(grad_vol), _ptr(P), _ptr(gP), _ptr(gxy), ws, n,
                                      _stream(stream)), "nursd_adjoint")
        return gP, gxy


def subsample_nearest(P: torch.Tensor, D: int, stream=None) -> torch.Tensor:
    """Compression preprocessing: keep the relay-grid phasors P [F][ny][nx] on
    the stride-D lattice and fill every point from its nearest kept sample."""
    lib = _lib.load()
    if P.dim() != 3:
        raise ValueError("P must be [F][ny][nx]")
    _need(P, torch.complex64, tuple(P.shape), "P")
    out = torch.empty_like(P)
    check(lib.nursd_subsample_nearest(_ptr(P), _ptr(out), P.shape[0], P.shape[1], P.shape[2], int(D),
                                      _stream(stream)), "nursd_subsample_nearest")
    return out


class Batch:
    """Many GRID plans served by one captured graph of grouped persistent
    kernels (C handle nursd_batch).  The workspace is a torch allocation
    owned by this object; with autotune the first forward first times the
    candidate configurations (nursd_batch_autotune, which synchronises)."""

    def __init__(self, plans: list[Plan], autotune: bool = True, stream=None):
        self._lib = _lib.load()
        self.plans = list(plans)
        self.autotune = bool(autotune)
        self._tuned = False
        arr = (c_void_p * len(plans))(*[p.handle.value for p in plans])
        h = c_void_p()
        check(self._lib.nursd_batch_create(arr, len(plans), 1 if autotune else 0, _stream(stream), byref(h)),
              "nursd_batch_create")
        self.handle = h
        n = c_size_t()
        check(self._lib.nursd_batch_workspace_size(self.handle, byref(n)), "nursd_batch_workspace_size")
        self.workspace_bytes = n.value
        dev = plans[0].device
        self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=dev)
        base = self._ws.data_ptr()
        self._ws_ptr = base + (-base) % 256

    def __del__(self):
        if getattr(self, "handle", None):
            self._lib.nursd_batch_destroy(self.handle)
            self.handle = None

    def forward(self, hists: list[torch.Tensor], outs: list[torch.Tensor] | None = None, stream=None):
        if len(hists) != len(self.plans):
            raise ValueError("one histogram tensor per plan")
        if outs is None:
            outs = [torch.empty(p.out_shape(), dtype=torch.float32, device=p.device) for p in self.plans]
        for p, h, o in zip(self.plans, hists, outs):
            _need(h, torch.float32, (p.L, p.n_time), "hist")
            _need(o, torch.float32, p.out_shape(), "I")
        self._keep = (list(hists), list(outs))
        hp = (c_void_p * len(hists))(*[h.data_ptr() for h in hists])
        op = (c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        ws, n = c_void_p(self._ws_ptr), c_size_t(self.workspace_bytes)
        if self.autotune and not self._tuned:
            check(self._lib.nursd_batch_autotune(self.handle, hp, op, ws, n, _stream(stream)), "nursd_batch_autotune")
            self._tuned = True
        check(self._lib.nursd_batch_forward(self.handle, hp, op, ws, n, _stream(stream)), "nursd_batch_forward")
        return outs

    def info(self) -> dict:
        b, nl, nt = c_int32(), c_int32(), c_int32()
        tried = (c_int32 * 16)()
        tms = (ctypes.c_float * 16)()
        wsb = c_size_t()
        check(self._lib.nursd_batch_info(self.handle, byref(b), byref(nl), byref(nt), tried, tms, byref(wsb)),
              "nursd_batch_info")
        names = {0: "queue", 1: "static", 2: "flat"}
        serial = {0: "none", 1: "M>=256", 2: "M>=512"}

        def label(t):
            return (f"{names[(t // 1000) % 10]}/R{t % 1000}/serial:{serial[(t // 10000) % 10]}"
                    f"/shared:{t // 100000}")
        buf = ctypes.create_string_buffer(4096)
        check(self._lib.nursd_batch_tuning(self.handle, buf, len(buf)), "nursd_batch_tuning")
        kernels = [x for x in buf.value.decode().split("; ") if x]
        return {"rounds": b.value % 1000, "schedule": names[(b.value // 1000) % 10],
                "serial": serial[(b.value // 10000) % 10], "shared_kernels": b.value // 100000,
                "launches": nl.value, "workspace_bytes": wsb.value,
                "tried": {label(t): tms[i] for i, t in enumerate(tried[:nt.value])},
                "kernel_choices": kernels}


def plan_from_workload(w, device, relay_xy: torch.Tensor | None = None, **kw) -> Plan:
    """Plan for a workloads.scenes.Workload (relay positions copied to `device`)."""
    wl, g = w.wavelet, w.grid
    if relay_xy is None:
        relay_xy = torch.from_numpy(np.ascontiguousarray(w.relay_xy)).to(device)
    mode = {"grid": MODE_GRID, "points": MODE_POINTS, "srsd": MODE_SRSD, "srsd_points": MODE_SRSD_POINTS,
            "grid3d": MODE_GRID3D}[w.mode]
    extra = {}
    if w.mode in ("points", "srsd_points"):
        extra["plane_ptr"] = w.plane_ptr
        extra["voxel_xy"] = torch.from_numpy(np.ascontiguousarray(w.voxel_xy)).to(device)
    if w.mode in ("srsd", "srsd_points"):
        extra["zref"] = w.zref
    if w.mode == "grid3d":
        e = w.extra
        extra["relay_z"] = torch.from_numpy(np.ascontiguousarray(e["relay_z"], dtype=np.float32)).to(device)
        extra["z_mid"], extra["dz3"], extra["mz3"] = e["z_mid"], e.get("dz3", 0.0), e.get("mz3", 0)
    args = dict(lambda_c=wl.lambda_c, n_time=wl.n_time, dt=wl.dt, t0=wl.t0, n_freq=wl.n_freq, z=g.z,
                mode=mode, x0=g.x0, y0=g.y0, dx=g.dx, dy=g.dy, nx=g.nx, ny=g.ny, bins=wl.bins,
                sigma_rel=wl.sigma_rel, pad=w.pad, xp=tuple(w.xp))
    args.update(extra)
    args.update(kw)
    return Plan(relay_xy, **args)
