"""Python binding of ``libraymeta.so`` (the C ABI in ``include/raymeta.h``):
radar IF synthesis from ray meta data (Section II, Eqs. 1-7).

Argument marshalling only: every step (hit update, path lengths, antenna
displacement, delays, the IF sum, the range-Doppler transform, span masks)
runs in the HIP library.  torch provides device memory and the stream.  If
the library is missing this module raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libraymeta.so")

RMD_OK = 0
STATUS_NAMES = {0: "RMD_OK", -1: "RMD_EINVAL", -3: "RMD_EHIP", -8: "RMD_ESCENE"}
MAX_SAMPLES = 1024
MAX_FFT = 4096
MAX_RAYS = 1 << 30
SPAN_ANY, SPAN_NONE, SPAN_ALL = 0, 1, 2

# Every symbol include/raymeta.h declares (checked by the CPU test suite).
EXPORTED = ("rmd_api_version", "rmd_last_error", "rmd_check_scene", "rmd_workspace_bytes", "rmd_if_cube",
            "rmd_if_cube_static", "rmd_if_cube_direct", "rmd_range_doppler", "rmd_span_weights")
STATIC_SCRATCH_BYTES = 64 << 20   # RMD_STATIC_SCRATCH_BYTES
# Evaluation of the sum over rays: "spread" (type-1 non-uniform FFT,
# rmd_if_cube) or "direct" (term by term on the matrix cores, rmd_if_cube_direct).
METHODS = {"spread": "rmd_if_cube", "direct": "rmd_if_cube_direct"}


class Radar(C.Structure):
    _fields_ = [("f_c", C.c_double), ("bandwidth", C.c_double), ("t_chirp", C.c_double), ("f_s", C.c_double),
                ("n_samples", C.c_int32), ("n_chirps", C.c_int32)]


class Scene(C.Structure):
    _fields_ = [("n_meshes", C.c_int32), ("n_tris", C.c_int32), ("n_verts", C.c_int32), ("n_rays", C.c_int32),
                ("n_hits", C.c_int64),
                ("mesh_tri_off", C.c_void_p), ("tris", C.c_void_p), ("verts", C.c_void_p),
                ("ray_off", C.c_void_p), ("hit_mesh", C.c_void_p), ("hit_tri", C.c_void_p),
                ("hit_u", C.c_void_p), ("hit_v", C.c_void_p)]


class SpanRule(C.Structure):
    _fields_ = [("mode", C.c_int32), ("min_hits", C.c_int32), ("max_hits", C.c_int32)]


class RaymetaError(RuntimeError):
    def __init__(self, status, fn, msg):
        super().__init__(f"{fn} -> {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sigs = {
        "rmd_api_version": ([], C.c_int32),
        "rmd_last_error": ([], C.c_char_p),
        "rmd_check_scene": ([C.POINTER(Scene), C.c_int32, P, C.POINTER(C.c_int64), P], C.c_int32),
        "rmd_workspace_bytes": ([C.POINTER(Scene), C.POINTER(Radar), C.c_int32, C.c_int32, C.POINTER(C.c_int64)],
                                C.c_int32),
        "rmd_if_cube": ([C.POINTER(Scene), C.POINTER(Radar), C.c_int32, P, P, C.c_int32, C.c_int32, P, P,
                         C.c_int64, P], C.c_int32),
        "rmd_if_cube_direct": ([C.POINTER(Scene), C.POINTER(Radar), C.c_int32, P, P, C.c_int32, C.c_int32, P, P,
                                C.c_int64, P], C.c_int32),
        "rmd_if_cube_static": ([C.POINTER(Scene), C.POINTER(Radar), C.c_int32, P, P, C.c_int32, C.c_int32, P, P],
                               C.c_int32),
        "rmd_range_doppler": ([P, P, C.c_int32, C.c_int32, C.c_int32, P], C.c_int32),
        "rmd_span_weights": ([C.POINTER(Scene), P, C.POINTER(SpanRule), P, P, P], C.c_int32),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(status, fn):
    if status != RMD_OK:
        raise RaymetaError(status, fn, load().rmd_last_error().decode())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _device_array(x, dtype, n, name, device):
    """Check that a tensor handed to the library is a contiguous device array
    of `n` elements of `dtype` on `device` (the kernels read exactly n)."""
    import torch
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if x.dtype != dtype or not x.is_contiguous() or x.numel() != n or x.device != device:
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of {n} elements on {device}; "
                         f"got {x.dtype}, {tuple(x.shape)}, contiguous={x.is_contiguous()}, on {x.device}")
    return C.c_void_p(x.data_ptr())


def radar_struct(radar) -> Radar:
    return Radar(radar.f_c, radar.bandwidth, radar.t_chirp, radar.f_s, radar.n_samples, radar.n_chirps)


class DeviceScene:
    """A ``rayscene.RayScene`` resident in device memory (torch tensors) with
    its ``rmd_scene`` descriptor."""

    def __init__(self, scene, device="cuda"):
        import torch
        load()
        self.scene = scene
        self.radar = scene.radar
        self.device = torch.device(device)
        # The kernels range-check every index they read, but trust these sizes.
        nh, nr = scene.n_hits, scene.n_rays
        checks = [
            (np.shape(scene.ray_off) == (nr + 1,), "ray_off must have n_rays + 1 entries"),
            (all(np.shape(x) == (nh,) for x in (scene.hit_tri, scene.hit_u, scene.hit_v)),
             "hit_mesh, hit_tri, hit_u and hit_v must have the same length"),
            (np.ndim(scene.tris) == 2 and np.shape(scene.tris)[1] == 3, "tris must be [n_tris][3]"),
            (np.ndim(scene.verts) == 3 and np.shape(scene.verts)[0] == scene.radar.n_chirps
             and np.shape(scene.verts)[2] == 3, "verts must be [n_chirps][n_verts][3]"),
            (np.shape(scene.tx_virt) == np.shape(scene.rx_virt) and np.shape(scene.tx_virt)[1:] == (3,),
             "tx_virt and rx_virt must be [n_pairs][3]"),
            (scene.amp is None or np.shape(scene.amp) == (nr,), "amp must have n_rays entries"),
        ]
        for ok, msg in checks:
            if not ok:
                raise ValueError(msg)
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(self.device)   # noqa: E731
        self.mesh_tri_off = t(scene.mesh_tri_off, np.int32)
        self.device = self.mesh_tri_off.device          # with its index ("cuda" -> "cuda:0")
        self.tris = t(scene.tris, np.int32)
        self.verts = t(scene.verts, np.float64)
        self.ray_off = t(scene.ray_off, np.int32)
        self.hit_mesh = t(scene.hit_mesh, np.int32)
        self.hit_tri = t(scene.hit_tri, np.int32)
        self.hit_u = t(scene.hit_u, np.float32)
        self.hit_v = t(scene.hit_v, np.float32)
        self.pairs = t(np.concatenate([scene.tx_virt, scene.rx_virt], axis=1), np.float64)
        self.amp = None if scene.amp is None else t(scene.amp, np.float32)
        self.desc = Scene(scene.n_meshes, int(scene.tris.shape[0]), scene.n_verts, scene.n_rays, scene.n_hits,
                          self.mesh_tri_off.data_ptr(), self.tris.data_ptr(), self.verts.data_ptr(),
                          self.ray_off.data_ptr(), self.hit_mesh.data_ptr(), self.hit_tri.data_ptr(),
                          self.hit_u.data_ptr(), self.hit_v.data_ptr())

    @property
    def n_pairs(self):
        return int(self.pairs.shape[0])


def check_scene(ds: DeviceScene, stream=None) -> int:
    """Rays with out-of-range meta data (0 for a valid scene).  Synchronous."""
    import torch
    ws = torch.empty(1, dtype=torch.int64, device=ds.device)
    bad = C.c_int64(0)
    st = load().rmd_check_scene(C.byref(ds.desc), ds.radar.n_chirps, C.c_void_p(ws.data_ptr()), C.byref(bad),
                                _stream(stream))
    if st not in (RMD_OK, -8):
        check(st, "rmd_check_scene")
    return int(bad.value)


def workspace_bytes(ds: DeviceScene, n_pairs: int, chirp_count: int) -> int:
    out = C.c_int64(0)
    r = radar_struct(ds.radar)
    check(load().rmd_workspace_bytes(C.byref(ds.desc), C.byref(r), n_pairs, chirp_count, C.byref(out)),
          "rmd_workspace_bytes")
    return int(out.value)


class Synthesizer:
    """IF cubes of one device scene: owns the output and workspace buffers for
    a chirp-block size, so repeated calls allocate nothing."""

    def __init__(self, ds: DeviceScene, chirp_count: Optional[int] = None, pairs=None, method: str = "spread"):
        import torch
        if method not in METHODS:
            raise ValueError(f"method must be one of {sorted(METHODS)}")
        self.fn = METHODS[method]
        self.ds = ds
        self.pairs = ds.pairs if pairs is None else torch.as_tensor(np.asarray(pairs, np.float64)).to(ds.device)
        if self.pairs.dim() != 2 or self.pairs.shape[1] != 6:
            raise ValueError("pairs must be [n_pairs][6]: x'_tx then x'_rx of each pair")
        self.pairs = self.pairs.contiguous()
        self.n_pairs = int(self.pairs.shape[0])
        self.chirp_count = chirp_count or ds.radar.n_chirps
        self.radar = radar_struct(ds.radar)
        nbytes = workspace_bytes(ds, self.n_pairs, self.chirp_count)
        self.workspace = torch.empty(max(nbytes, 256) // 8 + 32, dtype=torch.float64, device=ds.device)
        self.out = torch.empty((self.n_pairs, self.chirp_count, ds.radar.n_samples), dtype=torch.complex64,
                               device=ds.device)
        self.ws_bytes = nbytes

    def run(self, chirp0: int = 0, weights=None, stream=None):
        """s[q, j - chirp0, n] for chirps [chirp0, chirp0 + chirp_count); returns
        the (reused) output tensor, valid once the stream has run."""
        import torch
        wptr = None if weights is None else _device_array(weights, torch.float32, self.ds.scene.n_rays, "weights",
                                                          self.ds.device)
        check(getattr(load(), self.fn)(C.byref(self.ds.desc), C.byref(self.radar), self.n_pairs,
                                       C.c_void_p(self.pairs.data_ptr()), wptr, chirp0, self.chirp_count,
                                       C.c_void_p(self.out.data_ptr()), C.c_void_p(self.workspace.data_ptr()),
                                       self.workspace.numel() * 8, _stream(stream)), self.fn)
        return self.out


def if_cube(ds: DeviceScene, weights=None, chirps: Optional[Sequence[int]] = None, stream=None,
            method: str = "spread"):
    """The IF cube (Eqs. 1, 2, 3, 6, 7) as a new complex64 tensor [pair][chirp][sample]."""
    j0, j1 = (0, ds.radar.n_chirps) if chirps is None else (chirps[0], chirps[-1] + 1)
    if weights is None:
        weights = ds.amp
    syn = Synthesizer(ds, chirp_count=j1 - j0, method=method)
    return syn.run(j0, weights, stream).clone()


def range_doppler(s, out=None, stream=None):
    """Eq. 4 on a complex64 cube [pair][chirp][sample] (new tensor unless ``out``)."""
    import torch
    if not (isinstance(s, torch.Tensor) and s.dtype == torch.complex64 and s.is_contiguous() and s.dim() == 3
            and s.is_cuda):
        raise ValueError("s must be a contiguous complex64 device tensor [pair][chirp][sample]")
    out = torch.empty_like(s) if out is None else out
    _device_array(out, torch.complex64, s.numel(), "out", s.device)
    if out.shape != s.shape:
        raise ValueError("out must have the shape of s")
    check(load().rmd_range_doppler(C.c_void_p(s.data_ptr()), C.c_void_p(out.data_ptr()), s.shape[0], s.shape[1],
                                   s.shape[2], _stream(stream)), "rmd_range_doppler")
    return out


def span_weights(ds: DeviceScene, meshes=(), mode=SPAN_ANY, min_hits=1, max_hits=(1 << 31) - 1, amp="scene",
                 stream=None):
    """Eq. 5: per-ray weights of the rays a filter rule keeps (times A)."""
    import torch
    in_set = np.zeros(ds.scene.n_meshes, np.uint8)
    in_set[list(meshes)] = 1
    in_set = torch.from_numpy(in_set).to(ds.device)
    rule = SpanRule(mode, min_hits, max_hits)
    a = ds.amp if (isinstance(amp, str) and amp == "scene") else amp
    if a is not None:
        _device_array(a, torch.float32, ds.scene.n_rays, "amp", ds.device)
    w = torch.empty(ds.scene.n_rays, dtype=torch.float32, device=ds.device)
    check(load().rmd_span_weights(C.byref(ds.desc), C.c_void_p(in_set.data_ptr()), C.byref(rule),
                                  None if a is None else C.c_void_p(a.data_ptr()), C.c_void_p(w.data_ptr()),
                                  _stream(stream)), "rmd_span_weights")
    return w
