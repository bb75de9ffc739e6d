"""Seeded synthetic inputs for the Yee FDTD step.

This module only draws and lays out inputs (grids, material lattices, PEC
masks, source and probe positions, frequency lists, initial fields).  It holds
none of the update arithmetic: the time step, the update coefficients, the
CPML profiles and the source waveforms are computed separately by the HIP
library and by the FP64 oracle.  Both sides receive the same objects built
here, so no random-number parity is needed.

All random draws use ``numpy.random.Generator(PCG64(seed))``.

Workloads (no public dataset is involved; every input is synthetic):
  * ``plain_pec_box``          32^3 FP64 PEC box, centred 8^3 eps_r = 4 block,
                               Gaussian-derivative Ez source (t0 = 40 dt, tau = 12 dt),
                               4 seeded Ez probes, 200 steps.
  * ``waveguide_ports``        12 x 12 x 140 PEC waveguide, CPML on the z faces, for
                               two-run S-parameters (reference, PEC short, dielectric slab)
  * ``cpml_block_lattice``     256^3 FP32, 10-cell CPML on all faces, 8^3-cell block
                               lattice eps_r ~ U[1, 10), sigma ~ U[0, 0.1) S/m,
                               modulated-Gaussian Ez source at 10 GHz (dx = 0.5 mm),
                               16 probes, 64 DFT frequencies, 1000 steps.
  * ``fp16_substrate``         512 x 512 x 256, FP16 storage, 3 seeded dielectric
                               slabs (eps_r in {2.2, 4.4, 10.2}) with a PEC strip mask
                               on the top face, 2000 steps.
  * ``serving_request``        one request of the serving sweep (cubic side from
                               {32, 48, 64, 96, 128, 160}, 500-3000 steps, CPML 8).
  * ``adjoint_design``         128^3 FP32, CPML 10, per-cell design eps_r ~ U[1, 6) in
                               the central 64^3 region, 16 probes, 1024 steps.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

COMP_INDEX = {"Ex": 0, "Ey": 1, "Ez": 2, "Hx": 3, "Hy": 4, "Hz": 5}


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class SourceSpec:
    """Soft source on E component ``comp`` at (i, j, k).

    ``unit`` says how t0 and tau are given: "s" (seconds) or "dt" (multiples
    of the time step, resolved by each side with its own dt)."""
    comp: int
    i: int
    j: int
    k: int
    kind: str = "gauss_deriv"
    amp: float = 1.0
    t0: float = 0.0
    tau: float = 1.0
    f0: float = 0.0
    unit: str = "s"

    def times(self, dt: float) -> Tuple[float, float]:
        if self.unit == "dt":
            return self.t0 * dt, self.tau * dt
        return self.t0, self.tau


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    courant: float = 0.99
    precision: str = "f32"                 # "f64" | "f32" | "f16"
    cpml_cells: Tuple[int, int, int] = (0, 0, 0)
    cpml_m: float = 3.0
    cpml_sigma_max: Optional[float] = None  # None: per-axis default
    cpml_kappa_max: float = 1.0
    cpml_alpha_max: float = 0.0
    fp16_exp: Tuple[int, ...] = (0, 0, 0, 9, 9, 9)
    # rectilinear block lattice
    seg_x: np.ndarray = None
    seg_y: np.ndarray = None
    seg_z: np.ndarray = None
    eps_blk: np.ndarray = None              # flat [(bz*nsy + by)*nsx + bx]
    sig_blk: np.ndarray = None
    nsx: int = 1
    nsy: int = 1
    nsz: int = 1
    pec_planes: List[Tuple[int, np.ndarray]] = field(default_factory=list)  # (k, mask[ny, nx])
    pec_volume: Optional[np.ndarray] = None   # uint8 [nx, ny, nz]: bit 0 Ex, 1 Ey, 2 Ez held at zero
    sources: List[SourceSpec] = field(default_factory=list)
    probes: List[Tuple[int, int, int, int]] = field(default_factory=list)   # (comp, i, j, k)
    freqs: np.ndarray = field(default_factory=lambda: np.zeros(0))
    steps: int = 100
    design: Optional[Tuple[int, int]] = None  # [d0, d1) per axis of a gradient workload

    def __post_init__(self):
        if self.seg_x is None:
            self.seg_x = np.zeros(self.nx, np.int32)
            self.seg_y = np.zeros(self.ny, np.int32)
            self.seg_z = np.zeros(self.nz, np.int32)
            self.eps_blk = np.ones(1)
            self.sig_blk = np.zeros(1)
            self.nsx = self.nsy = self.nsz = 1

    # -- representation changes (indexing only) ------------------------------
    def cell_materials(self):
        """Per-cell (eps_r, sigma) arrays of shape (nx, ny, nz)."""
        idx = (self.seg_z[None, None, :] * self.nsy + self.seg_y[None, :, None]) * self.nsx \
            + self.seg_x[:, None, None]
        return self.eps_blk[idx], self.sig_blk[idx]

    def pec_component_masks(self):
        """PEC planes as boolean arrays of the E components' Yee shapes."""
        if not self.pec_planes and self.pec_volume is None:
            return None
        nx, ny, nz = self.nx, self.ny, self.nz
        out = {"Ex": np.zeros((nx, ny + 1, nz + 1), bool),
               "Ey": np.zeros((nx + 1, ny, nz + 1), bool),
               "Ez": np.zeros((nx + 1, ny + 1, nz), bool)}
        for k, m in self.pec_planes:
            mt = np.asarray(m).T  # (nx, ny)
            out["Ex"][:nx, :ny, k] |= (mt & 1) != 0
            out["Ey"][:nx, :ny, k] |= (mt & 2) != 0
            out["Ez"][:nx, :ny, k] |= (mt & 4) != 0
        if self.pec_volume is not None:
            v = np.asarray(self.pec_volume)
            out["Ex"][:nx, :ny, :nz] |= (v & 1) != 0
            out["Ey"][:nx, :ny, :nz] |= (v & 2) != 0
            out["Ez"][:nx, :ny, :nz] |= (v & 4) != 0
        return out

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def _segments(n: int, starts: Sequence[int]) -> np.ndarray:
    """Block index per cell for blocks beginning at the given start indices."""
    seg = np.zeros(n, np.int32)
    for b, s in enumerate(starts):
        seg[s:] = b
    return seg


def _interior_probes(rng, wl: Workload, count: int, comp: int = 2, margin: int = 1,
                     exclude=(), region=None) -> List[Tuple[int, int, int, int]]:
    """Distinct samples of ``comp`` drawn without replacement, outside the CPML
    plus ``margin`` cells and away from excluded points / an excluded box."""
    lo = [c + margin for c in wl.cpml_cells]
    hi = [n - c - margin for n, c in zip((wl.nx, wl.ny, wl.nz), wl.cpml_cells)]
    lo = [max(v, 1) for v in lo]
    out, seen = [], set(tuple(e) for e in exclude)
    tries = 0
    while len(out) < count:
        tries += 1
        if tries > 1000 * count:
            raise ValueError("no room for the requested probes")
        p = tuple(int(rng.integers(l, h)) for l, h in zip(lo, hi))
        if p in seen:
            continue
        if region is not None and all(region[a][0] <= p[a] < region[a][1] for a in range(3)):
            continue
        seen.add(p)
        out.append((comp,) + p)
    return out


def dft_frequencies(f0: float, n: int = 64) -> np.ndarray:
    """f_m = f0 (1/2 + m/(n-1)), m = 0..n-1 (the band f0/2 .. 3 f0/2)."""
    return f0 * (0.5 + np.arange(n) / (n - 1))


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------

def plain_pec_box(seed: int = 1) -> Workload:
    """32^3 cells, FP64, dx = 1 mm, PEC walls, eps_r = 4 on cells 12..19 per axis."""
    n = 32
    starts = [0, 12, 20]
    seg = _segments(n, starts)
    eps = np.ones(27)
    eps[(1 * 3 + 1) * 3 + 1] = 4.0
    wl = Workload("plain_pec_box_32", n, n, n, 1e-3, 1e-3, 1e-3, precision="f64",
                  seg_x=seg, seg_y=seg.copy(), seg_z=seg.copy(), eps_blk=eps, sig_blk=np.zeros(27),
                  nsx=3, nsy=3, nsz=3, steps=200)
    wl.sources = [SourceSpec(2, 16, 16, 16, "gauss_deriv", 1.0, 40.0, 12.0, unit="dt")]
    wl.probes = _interior_probes(rng_for(seed), wl, 4, exclude=[(16, 16, 16)])
    return wl


def cpml_block_lattice(n: int = 256, steps: int = 1000, seed: int = 2, precision: str = "f32",
                       cpml: int = 10, nprobes: int = 16, nfreq: int = 64, block: int = 8,
                       ny: Optional[int] = None, nz: Optional[int] = None) -> Workload:
    """The 256^3 FP32 CPML workload (sizes adjustable for tests)."""
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    rng = rng_for(seed)
    bx, by, bz = (n + block - 1) // block, (ny + block - 1) // block, (nz + block - 1) // block
    nb = bx * by * bz
    eps = rng.uniform(1.0, 10.0, nb)
    sig = rng.uniform(0.0, 0.1, nb)
    f0 = 10e9
    tau = 1.0 / (2.0 * f0)
    wl = Workload(f"cpml_block_lattice_{n}x{ny}x{nz}", n, ny, nz, 0.5e-3, 0.5e-3, 0.5e-3,
                  precision=precision, cpml_cells=(cpml, cpml, cpml),
                  seg_x=(np.arange(n) // block).astype(np.int32),
                  seg_y=(np.arange(ny) // block).astype(np.int32),
                  seg_z=(np.arange(nz) // block).astype(np.int32),
                  eps_blk=eps, sig_blk=sig, nsx=bx, nsy=by, nsz=bz, steps=steps)
    c = (n // 2, ny // 2, nz // 2)
    wl.sources = [SourceSpec(2, c[0], c[1], c[2], "mod_gauss", 1.0, 4 * tau, tau, f0, unit="s")]
    wl.probes = _interior_probes(rng, wl, nprobes, exclude=[c])
    wl.freqs = dft_frequencies(f0, nfreq)
    return wl


def fp16_substrate(nx: int = 512, ny: int = 512, nz: int = 256, steps: int = 2000, seed: int = 3,
                   cpml: int = 10) -> Workload:
    """Layered substrate with a PEC strip mask, FP16 storage (sizes adjustable)."""
    rng = rng_for(seed)
    zs = nz / 256.0
    xs = nx / 512.0
    thick = [max(2, int(round(t * zs))) for t in rng.integers(16, 49, 3)]
    perm = rng.permutation([2.2, 4.4, 10.2])
    k_base = cpml
    starts = [0, k_base, k_base + thick[0], k_base + thick[0] + thick[1]]
    k_top = starts[-1] + thick[2]
    starts.append(k_top)
    seg_z = _segments(nz, starts)
    eps = np.array([1.0, perm[0], perm[1], perm[2], 1.0])
    # FP16 storage scales (reading R17): E is stored as fp16(E * 2^12), H as
    # fp16(H * 2^21).  With a source of amplitude 1 V/m the fields stay below
    # 65504 / 2^12 = 16 V/m, and the far fields, down to ~1e-8 V/m, stay in
    # fp16's normal range (2^-14 / 2^12 = 1.5e-8) instead of its subnormals;
    # 2^9 is about eta0 * 1.36, so H * 2^21 spans the range E * 2^12 does.
    wl = Workload(f"fp16_substrate_{nx}x{ny}x{nz}", nx, ny, nz, 0.5e-3, 0.5e-3, 0.5e-3, precision="f16",
                  fp16_exp=(12, 12, 12, 21, 21, 21),
                  cpml_cells=(cpml, cpml, cpml), seg_x=np.zeros(nx, np.int32), seg_y=np.zeros(ny, np.int32),
                  seg_z=seg_z, eps_blk=eps, sig_blk=np.zeros(5), nsx=1, nsy=1, nsz=5, steps=steps)
    mask = np.zeros((ny, nx), np.uint8)
    strips = []
    lo, hix, hiy = cpml + 2, nx - cpml - 2, ny - cpml - 2
    for s in range(16):
        width = max(1, int(round(rng.integers(2, 9) * xs)))
        length = max(4, int(round(rng.integers(64, 449) * xs)))
        horiz = bool(rng.integers(0, 2))
        if horiz:
            length = min(length, hix - lo - 1)
            i0 = int(rng.integers(lo, hix - length))
            j0 = int(rng.integers(lo, hiy - width))
            mask[j0:j0 + width, i0:i0 + length] |= 3
            strips.append((i0 + length // 2, j0 + width // 2))
        else:
            length = min(length, hiy - lo - 1)
            i0 = int(rng.integers(lo, hix - width))
            j0 = int(rng.integers(lo, hiy - length))
            mask[j0:j0 + length, i0:i0 + width] |= 3
            strips.append((i0 + width // 2, j0 + length // 2))
    wl.pec_planes = [(k_top, mask)]
    f0 = 10e9
    tau = 1.0 / (2.0 * f0)
    si, sj = strips[0]
    wl.sources = [SourceSpec(2, si, sj, k_top - 1, "mod_gauss", 1.0, 4 * tau, tau, f0, unit="s")]
    probes = []
    prng = rng
    while len(probes) < 16:
        p = (2, int(prng.integers(lo, hix)), int(prng.integers(lo, hiy)),
             int(prng.integers(k_top + 1, max(k_top + 2, nz - cpml - 1))))
        if p not in probes:
            probes.append(p)
    wl.probes = probes
    wl.freqs = dft_frequencies(f0, 64)
    return wl


SERVING_SIDES = (32, 48, 64, 96, 128, 160)


def waveguide_ports(kind: str = "ref", precision: str = "f32", steps: int = 6000, n: int = 12, nz: int = 140,
                    cpml: int = 10) -> Workload:
    """A rectangular PEC waveguide along z (n x n cells of 0.5 mm, CPML only on
    the z faces) fed by a centred Ez point source, for two-run S-parameters.
    The source excites TM11 (cutoff 35.3 GHz for n = 12) and, by symmetry, no
    TM21/TM12; the next excited modes (TM13, TM31) are cut off below 79 GHz, so
    44-66 GHz carries one mode.  Port 0 is the Ez probe on the axis at k = 60,
    port 1 the one at k = 110.
      kind "ref":   the uniform guide (the incident wave);
      kind "short": a PEC plane (tangential E = 0) across the guide at k = 90;
      kind "slab":  a lossless eps_r = 2.5 slab filling k in [80, 88)."""
    d = 0.5e-3
    wl = Workload(f"waveguide_{kind}_{n}x{n}x{nz}", n, n, nz, d, d, d, precision=precision,
                  cpml_cells=(0, 0, cpml))
    tau, f0 = 30e-12, 55e9
    wl.sources = [SourceSpec(2, n // 2, n // 2, cpml + 4, "mod_gauss", 1.0, 4 * tau, tau, f0, unit="s")]
    wl.probes = [(2, n // 2, n // 2, 60), (2, n // 2, n // 2, 110)]
    wl.freqs = np.linspace(44e9, 66e9, 12)
    wl.steps = steps
    if kind == "short":
        wl.pec_planes = [(90, np.full((n, n), 3, np.int32))]
    elif kind == "slab":
        seg = np.zeros(nz, np.int32)
        seg[80:88] = 1
        wl.seg_z, wl.nsz = seg, 2
        wl.eps_blk, wl.sig_blk = np.array([1.0, 2.5]), np.zeros(2)
    elif kind != "ref":
        raise ValueError(f"unknown waveguide kind {kind!r}")
    return wl


def serving_request(seed: int, side: Optional[int] = None, steps: Optional[int] = None) -> Workload:
    """One serving request: cubic grid, eps_r ~ U[1, 12) on 8^3 blocks, CPML 8, FP32."""
    rng = rng_for(seed)
    side = int(rng.choice(SERVING_SIDES)) if side is None else side
    steps = int(rng.integers(500, 3001)) if steps is None else steps
    wl = cpml_block_lattice(n=side, steps=steps, seed=seed, cpml=8, nprobes=4, nfreq=16, block=8)
    nb = wl.nsx * wl.nsy * wl.nsz
    wl.eps_blk = rng_for(seed + 10_000).uniform(1.0, 12.0, nb)
    wl.sig_blk = np.zeros(nb)
    wl.name = f"serving_request_{side}"
    return wl


def serving_sweep(n_requests: int = 512, seed: int = 4):
    """(arrival offsets in units of the mean inter-arrival time, requests)."""
    rng = rng_for(seed)
    gaps = rng.exponential(1.0, n_requests)
    seeds = rng.integers(0, 2 ** 31 - 1, n_requests)
    return np.cumsum(gaps), [serving_request(int(s)) for s in seeds]


def adjoint_design(n: int = 128, design: Tuple[int, int] = (32, 96), steps: int = 1024, seed: int = 5,
                   cpml: int = 10, nprobes: int = 16) -> Workload:
    """Per-cell design eps_r ~ U[1, 6) on [d0, d1)^3, vacuum elsewhere."""
    rng = rng_for(seed)
    d0, d1 = design
    nd = d1 - d0
    # lattice: one segment below, one per design cell, one above (per axis)
    seg = np.zeros(n, np.int32)
    seg[d0:d1] = 1 + np.arange(nd)
    seg[d1:] = nd + 1
    ns = nd + 2
    eps = np.ones(ns ** 3)
    de = rng.uniform(1.0, 6.0, (nd, nd, nd))          # indexed [i, j, k]
    bz, by, bx = np.meshgrid(np.arange(nd) + 1, np.arange(nd) + 1, np.arange(nd) + 1, indexing="ij")
    eps[((bz * ns + by) * ns + bx).ravel()] = np.transpose(de, (2, 1, 0)).ravel()
    f0 = 10e9
    tau = 1.0 / (2.0 * f0)
    wl = Workload(f"adjoint_design_{n}", n, n, n, 0.5e-3, 0.5e-3, 0.5e-3, precision="f32",
                  cpml_cells=(cpml, cpml, cpml), seg_x=seg, seg_y=seg.copy(), seg_z=seg.copy(),
                  eps_blk=eps, sig_blk=np.zeros(ns ** 3), nsx=ns, nsy=ns, nsz=ns, steps=steps)
    src = (min(20, n // 2 - 1), n // 2, n // 2)
    wl.sources = [SourceSpec(2, src[0], src[1], src[2], "mod_gauss", 1.0, 4 * tau, tau, f0, unit="s")]
    wl.probes = _interior_probes(rng, wl, nprobes, exclude=[src],
                                 region=((d0, d1), (d0, d1), (d0, d1)))
    wl.design = (d0, d1)
    return wl


def adjoint_case(seed: int, nx: int = 26, ny: int = 22, nz: int = 20, steps: int = 150,
                 precision: str = "f64", probes: str = "e", cpml: int = 3) -> Workload:
    """Small gradient case with every feature the adjoint transposes: graded
    CPML with kappa and alpha, non-cubic cells, a lossy 4-cell block lattice
    (eps_r ~ U[1, 6), sigma ~ U[0, 0.3) S/m), a PEC mask plane, two sources and
    probes of E components ("e": Ez, Ex, Ey, one sample probed twice) or of H
    components only ("h")."""
    rng = rng_for(seed)
    block = 4
    bx, by, bz = (nx + block - 1) // block, (ny + block - 1) // block, (nz + block - 1) // block
    nb = bx * by * bz
    seg = [np.arange(n, dtype=np.int32) // block for n in (nx, ny, nz)]
    wl = Workload(f"adjoint_case_{nx}x{ny}x{nz}_{probes}", nx, ny, nz, 1.0e-3, 1.1e-3, 0.9e-3, precision=precision,
                  cpml_cells=(cpml, cpml, cpml), cpml_kappa_max=1.6, cpml_alpha_max=0.03,
                  seg_x=seg[0], seg_y=seg[1], seg_z=seg[2], eps_blk=rng.uniform(1.0, 6.0, nb),
                  sig_blk=rng.uniform(0.0, 0.3, nb), nsx=bx, nsy=by, nsz=bz, steps=steps)
    kp = nz // 2 + 2
    mask = np.zeros((ny, nx), np.uint8)
    mask[ny // 3: ny // 3 + 3, nx // 4: nx // 4 + 6] = 3
    mask[2 * ny // 3, nx // 2: nx // 2 + 4] = 7
    wl.pec_planes = [(kp, mask)]
    f0 = 30e9
    tau = 1.0 / (2.0 * f0)
    wl.sources = [SourceSpec(2, nx // 2, ny // 2, nz // 2, "mod_gauss", 1.0, 3 * tau, tau, f0, unit="s"),
                  SourceSpec(0, cpml + 2, ny // 2 + 1, nz // 3, "gauss_deriv", 0.5, 10.0, 4.0, unit="dt")]
    if probes == "e":
        pts = _interior_probes(rng, wl, 3, comp=2, exclude=[(nx // 2, ny // 2, nz // 2)])
        pts += _interior_probes(rng, wl, 2, comp=0) + _interior_probes(rng, wl, 1, comp=1)
        pts.append(pts[0])
    else:
        pts = (_interior_probes(rng, wl, 2, comp=3) + _interior_probes(rng, wl, 2, comp=4)
               + _interior_probes(rng, wl, 1, comp=5))
        pts.append(pts[-1])
    wl.probes = pts
    return wl


def random_initial_fields(wl: Workload, seed: int, h_scale: float = 1.0 / 377.0):
    """Random E^0, H^{-1/2} on the stored samples (i < nx, j < ny, k < nz), with
    the PEC-wall E samples (tangential on the faces) and the wall-normal H
    samples set to 0.  Arrays have shape (nx, ny, nz), index order (i, j, k).

    E is standard normal and H is h_scale times standard normal.  For FP16
    storage both are scaled by min(1, 2^(10 - s_E)), s_E the largest E
    exponent: white noise of that size peaks near 8 sigma in E and 13 sigma
    (of its initial H spread) in H over the first steps, which stays about a
    factor 4 inside the fp16 range 65504 / 2^s for exponents with
    s_H - s_E = 9."""
    rng = rng_for(seed)
    nx, ny, nz = wl.nx, wl.ny, wl.nz
    scale = min(1.0, 2.0 ** (10 - max(wl.fp16_exp[:3]))) if wl.precision == "f16" else 1.0
    f = {c: scale * rng.standard_normal((nx, ny, nz)) for c in ("Ex", "Ey", "Ez")}
    for c in ("Hx", "Hy", "Hz"):
        f[c] = scale * h_scale * rng.standard_normal((nx, ny, nz))
    f["Ex"][:, 0, :] = 0; f["Ex"][:, :, 0] = 0
    f["Ey"][0, :, :] = 0; f["Ey"][:, :, 0] = 0
    f["Ez"][0, :, :] = 0; f["Ez"][:, 0, :] = 0
    f["Hx"][0] = 0
    f["Hy"][:, 0] = 0
    f["Hz"][:, :, 0] = 0
    return f
