"""Seeded synthetic inputs for ray-meta-data IF synthesis.

This module only draws and lays out inputs: animated triangle meshes (one
vertex snapshot per chirp), the ray meta data a ray tracer would have stored
(per ray, the ordered list of hits as mesh ID, triangle index and barycentric
coordinates u, v), the radar parameters and the antenna positions of a MIMO
array.  It holds none of the method's arithmetic: hit positions, path
lengths, antenna displacement, delays, the IF sum and the range-Doppler
transform are computed separately by the HIP library and by the FP64 oracle,
which both receive the objects built here.

All random draws use ``numpy.random.Generator(PCG64(seed))``.

Scenes (no measured data, mesh or tracer output is involved; every input is
synthetic, standing in for the pedestrian scene of the paper's results):
  * ``pedestrian_scene``  8 meshes x 4096 triangles (cylindrical body parts
                          5-20 m in front of the radar, each with a rigid
                          velocity up to 5 m/s and a sinusoidal limb swing),
                          2^20 rays with 1-4 hits drawn with probabilities
                          (0.6, 0.25, 0.1, 0.05), a 77 GHz FMCW radar (1 GHz
                          sweep over 51.2 us, 10 MHz sampling, 512 samples,
                          128 chirps every 60 us) and a 3 TX x 4 RX array.
Smaller instances of the same recipe serve the parity tests.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

SPEED_OF_LIGHT = 299792458.0


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Radar:
    """FMCW chirp-sequence parameters (Section II.A)."""
    f_c: float = 77e9            # carrier frequency [Hz]
    bandwidth: float = 1e9       # sweep bandwidth B [Hz]
    t_chirp: float = 51.2e-6     # chirp duration T_c [s]
    t_frame: float = 60e-6       # time between chirps T_d [s]
    f_s: float = 10e6            # IF sampling rate [Hz]; fast time t_n = n / f_s
    n_samples: int = 512         # samples per chirp
    n_chirps: int = 128          # chirps per sequence


@dataclass
class RayScene:
    name: str
    radar: Radar
    # Meshes: triangles of mesh a are tris[mesh_tri_off[a]:mesh_tri_off[a+1]],
    # each a row of three global vertex indices.
    mesh_tri_off: np.ndarray            # int32 (n_meshes + 1,)
    tris: np.ndarray                    # int32 (n_tris, 3)
    verts: np.ndarray                   # float64 (n_chirps, n_verts, 3): vertex positions at t = j T_d
    # Ray meta data, CSR: the hits of ray i are entries ray_off[i]:ray_off[i+1],
    # in the order the ray met them (first hit first).
    ray_off: np.ndarray                 # int32 (n_rays + 1,)
    hit_mesh: np.ndarray                # int32 (n_hits,)  mesh ID a_k
    hit_tri: np.ndarray                 # int32 (n_hits,)  triangle index b_k within mesh a_k
    hit_u: np.ndarray                   # float32 (n_hits,)
    hit_v: np.ndarray                   # float32 (n_hits,)
    # Antennas: the pair the rays were traced for, and the pairs to synthesise.
    x_tx: np.ndarray                    # float64 (3,)
    x_rx: np.ndarray                    # float64 (3,)
    tx_virt: np.ndarray                 # float64 (n_pairs, 3)
    rx_virt: np.ndarray                 # float64 (n_pairs, 3)
    amp: np.ndarray = field(default=None)   # float32 (n_rays,) antenna-pattern weight per ray

    @property
    def n_rays(self) -> int:
        return int(self.ray_off.shape[0] - 1)

    @property
    def n_hits(self) -> int:
        return int(self.hit_mesh.shape[0])

    @property
    def n_meshes(self) -> int:
        return int(self.mesh_tri_off.shape[0] - 1)

    @property
    def n_pairs(self) -> int:
        return int(self.tx_virt.shape[0])

    @property
    def n_verts(self) -> int:
        return int(self.verts.shape[1])

    def with_rays(self, k: int) -> "RayScene":
        """The same scene restricted to its first k rays."""
        e = int(self.ray_off[k])
        return RayScene(self.name + f"[rays :{k}]", self.radar, self.mesh_tri_off, self.tris, self.verts,
                        self.ray_off[:k + 1].copy(), self.hit_mesh[:e], self.hit_tri[:e], self.hit_u[:e],
                        self.hit_v[:e], self.x_tx, self.x_rx, self.tx_virt, self.rx_virt,
                        None if self.amp is None else self.amp[:k])

    def with_chirps(self, j0: int, j1: int) -> "RayScene":
        """The same scene restricted to chirps [j0, j1)."""
        r = Radar(**{**self.radar.__dict__, "n_chirps": j1 - j0})
        return RayScene(self.name + f"[chirps {j0}:{j1}]", r, self.mesh_tri_off, self.tris,
                        np.ascontiguousarray(self.verts[j0:j1]), self.ray_off, self.hit_mesh, self.hit_tri,
                        self.hit_u, self.hit_v, self.x_tx, self.x_rx, self.tx_virt, self.rx_virt, self.amp)


def cylinder_mesh(n_around: int, n_up: int) -> Tuple[np.ndarray, np.ndarray]:
    """Unit cylinder (radius 1, height 1, axis z) as a quad grid split into
    triangles: n_around * n_up * 2 triangles, n_around * (n_up + 1) vertices."""
    ang = 2 * np.pi * np.arange(n_around) / n_around
    zs = np.arange(n_up + 1) / n_up
    verts = np.stack([np.tile(np.cos(ang), n_up + 1), np.tile(np.sin(ang), n_up + 1),
                      np.repeat(zs, n_around)], axis=1)
    tris = []
    for r in range(n_up):
        for c in range(n_around):
            a = r * n_around + c
            b = r * n_around + (c + 1) % n_around
            tris.append((a, b, a + n_around))
            tris.append((b, b + n_around, a + n_around))
    return verts, np.asarray(tris, dtype=np.int32)


def mimo_array(x_tx: np.ndarray, x_rx: np.ndarray, n_tx: int, n_rx: int, wavelength: float):
    """Virtual pairs of an n_tx x n_rx MIMO array along y: RX elements lambda/2
    apart, TX elements n_rx * lambda/2 apart (a filled virtual aperture).  Pair
    q = t * n_rx + r; pair 0 is the traced pair itself."""
    tx = np.array([x_tx + np.array([0.0, t * n_rx * wavelength / 2, 0.0]) for t in range(n_tx)])
    rx = np.array([x_rx + np.array([0.0, r * wavelength / 2, 0.0]) for r in range(n_rx)])
    tv = np.repeat(tx, n_rx, axis=0)
    rv = np.tile(rx, (n_tx, 1))
    return tv, rv


def random_hits(rng, n_rays: int, mesh_tri_off: np.ndarray, probs=(0.6, 0.25, 0.1, 0.05)):
    """Ray meta data: per ray 1..len(probs) hits with the given probabilities,
    each on a uniformly drawn mesh and triangle, at a uniform point of it."""
    counts = rng.choice(np.arange(1, len(probs) + 1), size=n_rays, p=np.asarray(probs) / np.sum(probs))
    ray_off = np.zeros(n_rays + 1, dtype=np.int64)
    np.cumsum(counts, out=ray_off[1:])
    n_hits = int(ray_off[-1])
    n_meshes = mesh_tri_off.shape[0] - 1
    hit_mesh = rng.integers(0, n_meshes, size=n_hits)
    sizes = np.diff(mesh_tri_off)
    hit_tri = np.floor(rng.random(n_hits) * sizes[hit_mesh]).astype(np.int64)
    u = rng.random(n_hits)
    v = rng.random(n_hits)
    fold = u + v > 1.0
    u[fold], v[fold] = 1.0 - u[fold], 1.0 - v[fold]
    return (ray_off.astype(np.int32), hit_mesh.astype(np.int32), hit_tri.astype(np.int32),
            u.astype(np.float32), v.astype(np.float32))


def pedestrian_scene(n_rays: int = 1 << 20, n_meshes: int = 8, tris_per_mesh: int = 4096,
                     radar: Optional[Radar] = None, n_tx: int = 3, n_rx: int = 4, seed: int = 6,
                     max_speed: float = 5.0) -> RayScene:
    """Body-part cylinders in front of the radar, animated over the chirps.

    Mesh a: radius 0.05-0.25 m, height 0.3-0.9 m, centred 5-20 m along x,
    |y| < 2 m, base 0-1.2 m.  Motion at t = j T_d: a rigid velocity (|v| up
    to ``max_speed``) plus a swing of up to 0.6 rad at 0.5-2 Hz about the
    mesh's top (a limb), so every mesh moves non-rigidly relative to the
    others."""
    radar = radar or Radar()
    rng = rng_for(seed)
    n_up = max(1, tris_per_mesh // 128)
    n_around = max(3, tris_per_mesh // (2 * n_up))
    base_v, base_t = cylinder_mesh(n_around, n_up)
    nv = base_v.shape[0]
    verts_local = []
    tris = []
    for a in range(n_meshes):
        r = rng.uniform(0.05, 0.25)
        h = rng.uniform(0.3, 0.9)
        verts_local.append(base_v * np.array([r, r, h]))
        tris.append(base_t + a * nv)
    tri_counts = [t.shape[0] for t in tris]
    mesh_tri_off = np.zeros(n_meshes + 1, dtype=np.int32)
    mesh_tri_off[1:] = np.cumsum(tri_counts)
    tris = np.concatenate(tris).astype(np.int32)

    centre = np.stack([rng.uniform(5.0, 20.0, n_meshes), rng.uniform(-2.0, 2.0, n_meshes),
                       rng.uniform(0.0, 1.2, n_meshes)], axis=1)
    vel_dir = rng.normal(size=(n_meshes, 3))
    vel = vel_dir / np.linalg.norm(vel_dir, axis=1, keepdims=True) * rng.uniform(0, max_speed, (n_meshes, 1))
    swing = rng.uniform(0.0, 0.6, n_meshes)
    freq = rng.uniform(0.5, 2.0, n_meshes)
    phase0 = rng.uniform(0, 2 * np.pi, n_meshes)

    verts = np.empty((radar.n_chirps, n_meshes * nv, 3))
    for j in range(radar.n_chirps):
        t = j * radar.t_frame
        for a in range(n_meshes):
            loc = verts_local[a]
            pivot = np.array([0.0, 0.0, loc[:, 2].max()])
            ang = swing[a] * np.sin(2 * np.pi * freq[a] * t + phase0[a])
            c, s = np.cos(ang), np.sin(ang)
            rot = np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])   # swing about x
            verts[j, a * nv:(a + 1) * nv] = (loc - pivot) @ rot.T + pivot + centre[a] + vel[a] * t

    ray_off, hit_mesh, hit_tri, u, v = random_hits(rng, n_rays, mesh_tri_off)
    wavelength = SPEED_OF_LIGHT / radar.f_c
    x_tx = np.array([0.0, -0.01, 0.5])
    x_rx = np.array([0.0, 0.01, 0.5])
    tx_virt, rx_virt = mimo_array(x_tx, x_rx, n_tx, n_rx, wavelength)
    return RayScene(f"pedestrian_{n_meshes}x{tris_per_mesh}_{n_rays}rays", radar, mesh_tri_off, tris,
                    verts, ray_off, hit_mesh, hit_tri, u, v, x_tx, x_rx, tx_virt, rx_virt,
                    np.ones(n_rays, dtype=np.float32))


def small_scene(n_rays: int = 4096, n_chirps: int = 8, n_samples: int = 256, n_tx: int = 2, n_rx: int = 2,
                seed: int = 7, tris_per_mesh: int = 256, n_meshes: int = 3) -> RayScene:
    """A parity-test instance of the same recipe."""
    radar = Radar(n_samples=n_samples, n_chirps=n_chirps)
    return pedestrian_scene(n_rays=n_rays, n_meshes=n_meshes, tris_per_mesh=tris_per_mesh, radar=radar,
                            n_tx=n_tx, n_rx=n_rx, seed=seed)


def random_amplitudes(scene: RayScene, seed: int) -> np.ndarray:
    """Per-ray pattern weights A in [0.2, 1) (the default is A = 1)."""
    return rng_for(seed).uniform(0.2, 1.0, scene.n_rays).astype(np.float32)
