"""Python binding of one Yee FDTD context (argument marshalling only).

PyTorch provides the device memory (one workspace tensor per context) and the
stream; every step of the update runs in ``libyee.so``.  Field arrays on the
Python side use index order (i, j, k) and shape (nx, ny, nz): the stored Yee
samples with i < nx, j < ny, k < nz (the samples outside are PEC-wall E or
wall-normal H samples and are identically zero).
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _lib
from .workloads import COMP_INDEX, Workload

_dp = C.POINTER(C.c_double)


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class YeeSolver:
    """A configured, bound and reset context for one workload on one device."""

    # byte the guard bands of a debug workspace are filled with
    GUARD_BYTE = 0xA5

    def __init__(self, wl: Workload, device: str = "cuda:0", series_len: Optional[int] = None,
                 tile_rows: int = 0, chunk_planes: int = 0, samples_per_lane: int = 0, stream=None,
                 steps_per_sweep: int = 0, sweep_rows: int = 0, sweep_planes: int = 0, guard_bytes: int = 0):
        """guard_bytes > 0 (debug): the workspace gets guard bands of at least
        that many bytes on both sides, filled with GUARD_BYTE; check_guards()
        tells whether any kernel wrote outside the footprint."""
        import torch
        self.torch = torch
        self.lib = _lib.load()
        self.wl = wl
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise RuntimeError("YeeSolver needs a GPU device (the HIP library has no CPU path)")
        d = _lib.GridDesc()
        d.nx, d.ny, d.nz = wl.nx, wl.ny, wl.nz
        d.dx, d.dy, d.dz = wl.dx, wl.dy, wl.dz
        d.courant = wl.courant
        d.precision = _lib.PRECISIONS[wl.precision]
        for q in range(3):
            d.cpml_cells[q] = int(wl.cpml_cells[q])
        d.cpml_m = wl.cpml_m
        d.cpml_sigma_max = -1.0 if wl.cpml_sigma_max is None else float(wl.cpml_sigma_max)
        d.cpml_kappa_max = wl.cpml_kappa_max
        d.cpml_alpha_max = wl.cpml_alpha_max
        for q in range(6):
            d.fp16_exp[q] = int(wl.fp16_exp[q])
        d.series_len = int(series_len if series_len is not None else max(1, wl.steps))
        self.desc = d
        ctx = C.c_void_p()
        _lib.check(self.lib.yee_create(C.byref(d), C.byref(ctx)), "yee_create")
        self.ctx = ctx
        dt = C.c_double()
        _lib.check(self.lib.yee_time_step(ctx, C.byref(dt)), "yee_time_step")
        self.dt = dt.value
        self._configure()
        nbytes = C.c_int64()
        _lib.check(self.lib.yee_footprint(ctx, C.byref(nbytes)), "yee_footprint")
        self.footprint = nbytes.value
        g = int(guard_bytes)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.footprint + 256 + 2 * g, dtype=torch.uint8, device=self.device)
            if g:
                self.workspace.fill_(self.GUARD_BYTE)
        base = self.workspace.data_ptr()
        aligned = (base + g + 255) & ~255
        self._ws_off = aligned - base
        self.guard_bytes = g
        _lib.check(self.lib.yee_bind_workspace(ctx, C.c_void_p(aligned), self.footprint), "yee_bind_workspace")
        if tile_rows or chunk_planes or samples_per_lane:
            _lib.check(self.lib.yee_set_launch(ctx, tile_rows, chunk_planes, samples_per_lane), "yee_set_launch")
        if steps_per_sweep or sweep_rows or sweep_planes:
            self.set_time_blocking(steps_per_sweep, sweep_rows, sweep_planes)
        self.stream = stream
        self.reset()

    # -- configuration ---------------------------------------------------------
    def _configure(self):
        wl, lib, ctx = self.wl, self.lib, self.ctx
        segx = np.ascontiguousarray(wl.seg_x, np.int32)
        segy = np.ascontiguousarray(wl.seg_y, np.int32)
        segz = np.ascontiguousarray(wl.seg_z, np.int32)
        eps = np.ascontiguousarray(wl.eps_blk, np.float64)
        sig = np.ascontiguousarray(wl.sig_blk, np.float64)
        _lib.check(lib.yee_set_materials(ctx, wl.nsx, wl.nsy, wl.nsz, _ptr(segx, C.c_int32), _ptr(segy, C.c_int32),
                                         _ptr(segz, C.c_int32), _ptr(eps, C.c_double), _ptr(sig, C.c_double)),
                   "yee_set_materials")
        for k, mask in wl.pec_planes:
            m = np.ascontiguousarray(mask, np.uint8)
            _lib.check(lib.yee_add_pec_plane(ctx, int(k), _ptr(m, C.c_uint8)), "yee_add_pec_plane")
        if wl.pec_volume is not None:
            v = np.ascontiguousarray(np.transpose(np.asarray(wl.pec_volume, np.uint8), (2, 1, 0)))
            _lib.check(lib.yee_set_pec_mask(ctx, _ptr(v, C.c_uint8)), "yee_set_pec_mask")
        for s in wl.sources:
            t0, tau = s.times(self.dt)
            sd = _lib.SourceDesc(s.comp, s.i, s.j, s.k, _lib.WAVEFORMS[s.kind], s.amp, t0, tau, s.f0)
            _lib.check(lib.yee_add_source(ctx, C.byref(sd)), "yee_add_source")
        for (comp, i, j, k) in wl.probes:
            pid = C.c_int32()
            _lib.check(lib.yee_add_probe(ctx, comp, i, j, k, C.byref(pid)), "yee_add_probe")
        f = np.ascontiguousarray(wl.freqs, np.float64)
        _lib.check(lib.yee_set_dft_freqs(ctx, _ptr(f, C.c_double) if f.size else None, int(f.size)),
                   "yee_set_dft_freqs")

    def _s(self):
        if self.stream is not None:
            return C.c_void_p(self.stream.cuda_stream)
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    # -- state -----------------------------------------------------------------
    def reset(self):
        _lib.check(self.lib.yee_reset(self.ctx, self._s()), "yee_reset")

    def set_materials(self, eps_blk: np.ndarray, sig_blk: Optional[np.ndarray] = None):
        """Replace the block values (same lattice) and upload them."""
        wl = self.wl
        eps = np.ascontiguousarray(eps_blk, np.float64)
        sig = np.ascontiguousarray(wl.sig_blk if sig_blk is None else sig_blk, np.float64)
        segx = np.ascontiguousarray(wl.seg_x, np.int32)
        segy = np.ascontiguousarray(wl.seg_y, np.int32)
        segz = np.ascontiguousarray(wl.seg_z, np.int32)
        _lib.check(self.lib.yee_set_materials(self.ctx, wl.nsx, wl.nsy, wl.nsz, _ptr(segx, C.c_int32),
                                              _ptr(segy, C.c_int32), _ptr(segz, C.c_int32),
                                              _ptr(eps, C.c_double), _ptr(sig, C.c_double)), "yee_set_materials")
        _lib.check(self.lib.yee_upload_materials(self.ctx, self._s()), "yee_upload_materials")

    def set_field(self, comp, arr: np.ndarray):
        ci = COMP_INDEX[comp] if isinstance(comp, str) else int(comp)
        a = np.ascontiguousarray(np.transpose(np.asarray(arr, np.float64), (2, 1, 0)))
        _lib.check(self.lib.yee_set_field(self.ctx, ci, _ptr(a, C.c_double), self._s()), "yee_set_field")

    def set_launch(self, tile_rows: int = 0, chunk_planes: int = 0, samples_per_lane: int = 0):
        """Launch shape of the fused step kernel (0 = automatic)."""
        _lib.check(self.lib.yee_set_launch(self.ctx, int(tile_rows), int(chunk_planes), int(samples_per_lane)),
                   "yee_set_launch")

    def set_time_blocking(self, steps_per_sweep: int = 0, tile_rows: int = 0, chunk_planes: int = 0):
        """Steps per sweep of yee_step (0 automatic, 1 single steps, 2 two-step
        sweeps) and the two-step launch shape (0 = automatic)."""
        _lib.check(self.lib.yee_set_time_blocking(self.ctx, int(steps_per_sweep), int(tile_rows), int(chunk_planes)),
                   "yee_set_time_blocking")

    def launch_info(self) -> dict:
        """The launch yee_step uses: steps per sweep, tile rows, chunk planes, samples per lane."""
        v = [C.c_int32() for _ in range(4)]
        _lib.check(self.lib.yee_launch_info(self.ctx, *[C.byref(x) for x in v]), "yee_launch_info")
        return dict(zip(("steps_per_sweep", "tile_rows", "chunk_planes", "samples_per_lane"), (x.value for x in v)))

    def step(self, n: int):
        _lib.check(self.lib.yee_step(self.ctx, int(n), self._s()), "yee_step")

    @property
    def steps_done(self) -> int:
        v = C.c_int64()
        _lib.check(self.lib.yee_steps_done(self.ctx, C.byref(v)), "yee_steps_done")
        return v.value

    def field(self, comp) -> np.ndarray:
        ci = COMP_INDEX[comp] if isinstance(comp, str) else int(comp)
        wl = self.wl
        out = np.empty((wl.nz, wl.ny, wl.nx), np.float64)
        _lib.check(self.lib.yee_read_field(self.ctx, ci, _ptr(out, C.c_double), self._s()), "yee_read_field")
        return np.ascontiguousarray(np.transpose(out, (2, 1, 0)))

    def series(self, first: int = 1, count: Optional[int] = None) -> np.ndarray:
        """Probe samples y[n], n = first .. first+count-1, as [count, n_probes]."""
        count = self.steps_done - first + 1 if count is None else count
        out = np.empty((max(count, 0), len(self.wl.probes)), np.float64)
        _lib.check(self.lib.yee_read_series(self.ctx, int(first), int(count),
                                            _ptr(out, C.c_double) if out.size else None, self._s()),
                   "yee_read_series")
        return out

    def dft(self) -> np.ndarray:
        npr, nf = len(self.wl.probes), len(self.wl.freqs)
        re = np.zeros((npr, nf))
        im = np.zeros((npr, nf))
        if npr and nf:
            _lib.check(self.lib.yee_read_dft(self.ctx, _ptr(re, C.c_double), _ptr(im, C.c_double), self._s()),
                       "yee_read_dft")
        return re + 1j * im

    # -- debug checks ------------------------------------------------------------
    def check_guards(self) -> bool:
        """True if both guard bands still hold GUARD_BYTE (needs guard_bytes > 0)."""
        if not self.guard_bytes:
            raise RuntimeError("no guard bands: create the solver with guard_bytes > 0")
        self.torch.cuda.synchronize(self.device)
        lo = self.workspace[:self._ws_off]
        hi = self.workspace[self._ws_off + self.footprint:]
        return bool((lo == self.GUARD_BYTE).all().item() and (hi == self.GUARD_BYTE).all().item())

    def write_counts(self, steps: int = 1) -> np.ndarray:
        """Debug: run `steps` single steps counting every store of the output
        field set; returns counts as [6][nz + 1][ny][row_pitch] (uint32)."""
        stride, pitch = C.c_int64(), C.c_int32()
        _lib.check(self.lib.yee_debug_layout(self.ctx, C.byref(stride), C.byref(pitch)), "yee_debug_layout")
        n = 6 * stride.value
        counts = self.torch.zeros(n, dtype=self.torch.int32, device=self.device)
        _lib.check(self.lib.yee_debug_set_write_counts(self.ctx, C.c_void_p(counts.data_ptr()), n),
                   "yee_debug_set_write_counts")
        try:
            self.step(steps)
            self.torch.cuda.synchronize(self.device)
        finally:
            self.lib.yee_debug_set_write_counts(self.ctx, None, 0)
        wl = self.wl
        per = (wl.nz + 1) * wl.ny * pitch.value
        host = counts.cpu().numpy().view(np.uint32).reshape(6, stride.value)
        return host[:, :per].reshape(6, wl.nz + 1, wl.ny, pitch.value)

    # -- health and checkpoints ------------------------------------------------
    def status(self):
        """(status, flags) of yee_status_flags: status 0, YEE_ENUMERIC (-5) or
        YEE_EOVERFLOW (-7), with a message for the latter two; never raises for them."""
        f = C.c_uint32()
        st = self.lib.yee_status_flags(self.ctx, C.byref(f), self._s())
        if st not in (0, -5, -7):
            _lib.check(st, "yee_status_flags")
        msg = self.lib.yee_last_error().decode(errors="replace") if st else ""
        return st, f.value, msg

    def state_bytes(self) -> int:
        v = C.c_int64()
        _lib.check(self.lib.yee_state_bytes(self.ctx, C.byref(v)), "yee_state_bytes")
        return v.value

    def save_state(self, out=None):
        """Device copy of the run's state (a uint8 tensor of state_bytes())."""
        n = self.state_bytes()
        if out is None:
            out = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        _lib.check(self.lib.yee_save_state(self.ctx, C.c_void_p(out.data_ptr()), int(out.numel()), self._s()),
                   "yee_save_state")
        return out

    def load_state(self, state):
        _lib.check(self.lib.yee_load_state(self.ctx, C.c_void_p(state.data_ptr()), int(state.numel()), self._s()),
                   "yee_load_state")

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.yee_destroy(self.ctx)
            self.ctx = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
