"""Plain FP64 numpy implementation of the 3-D Yee FDTD scheme.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

What is computed (the paper is silent on all of it; textbook definitions):

* Staggering and leapfrog (Yee 1966).  With (i, j, k) integer indices the
  six components sit at
      Ex ((i+1/2)dx, j dy, k dz)      shape (Nx,   Ny+1, Nz+1)
      Ey (i dx, (j+1/2)dy, k dz)      shape (Nx+1, Ny,   Nz+1)
      Ez (i dx, j dy, (k+1/2)dz)      shape (Nx+1, Ny+1, Nz  )
      Hx (i dx, (j+1/2)dy, (k+1/2)dz) shape (Nx+1, Ny,   Nz  )
      Hy ((i+1/2)dx, j dy, (k+1/2)dz) shape (Nx,   Ny+1, Nz  )
      Hz ((i+1/2)dx, (j+1/2)dy, k dz) shape (Nx,   Ny,   Nz+1)
  One step maps (E^n, H^{n-1/2}) to (E^{n+1}, H^{n+1/2}): first the H
  half-step with forward differences of E^n, then the E half-step with
  backward differences of H^{n+1/2}.
* Lossy E update with the semi-implicit conduction term (Taflove & Hagness,
  ch. 3):  Ca = (1 - s)/(1 + s),  Cb = (dt/eps)/(1 + s),  s = sigma dt/(2 eps),
  eps = eps0 eps_r.  mu_r = 1 everywhere, no magnetic loss.
* PEC: tangential E on the six outer faces is never updated (stays 0);
  a masked E sample has Ca = Cb = 0.
* CPML (Roden & Gedney 2000): inside the absorbing layer of axis w every
  difference d_w F of an update becomes d_w F / kappa_w + psi, where the
  auxiliary psi is first advanced, psi <- b_w psi + a_w d_w F, and then used.
* Soft sources add amp * w((n+1) dt) to one E sample after the E update.
* Probes record a component after the step; the running DFT accumulates
  X(f) += y^{n+1} exp(-i 2 pi f (n+1) dt) dt in FP64.
* Optional storage emulation: each stored component is rounded once per step
  (H after the H update, E after the E update and the source injection), as
  x <- fp16_RNE(x 2^s) 2^-s (FP16 storage) or x <- fp32_RNE(x) (FP32
  storage).
* Arithmetic: FP64 by default.  With arith="f32" every stored array (fields,
  CPML auxiliaries), the material coefficients and the CPML profiles are
  float32 and every operation of the step is a float32 operation (numpy keeps
  float32 when a Python float meets a float32 array); sources are evaluated
  in FP64 and added in float32, probes and the DFT stay FP64.  This is the
  arithmetic of the FP32 and FP16-storage modes of the device path, with the
  textbook operation order (no fused multiply-adds), so the two differ in
  the last bit of some results.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

# Physical constants: c0 exact, mu0 = 4 pi 1e-7, eps0 = 1/(mu0 c0^2), so that
# c0 = 1/sqrt(mu0 eps0) holds to rounding.
C0 = 299792458.0
MU0 = 4.0e-7 * np.pi
EPS0 = 1.0 / (MU0 * C0 * C0)
ETA0 = float(np.sqrt(MU0 / EPS0))

E_COMPONENTS = ("Ex", "Ey", "Ez")
H_COMPONENTS = ("Hx", "Hy", "Hz")
COMPONENTS = E_COMPONENTS + H_COMPONENTS


def yee_shape(comp: str, nx: int, ny: int, nz: int):
    """Exact array shape of one Yee component (index order i, j, k)."""
    return {
        "Ex": (nx, ny + 1, nz + 1),
        "Ey": (nx + 1, ny, nz + 1),
        "Ez": (nx + 1, ny + 1, nz),
        "Hx": (nx + 1, ny, nz),
        "Hy": (nx, ny + 1, nz),
        "Hz": (nx, ny, nz + 1),
    }[comp]


def time_step(dx: float, dy: float, dz: float, courant: float) -> float:
    """dt = S times the 3-D Courant limit 1/(c0 sqrt(dx^-2 + dy^-2 + dz^-2))."""
    return courant / (C0 * np.sqrt(1.0 / dx ** 2 + 1.0 / dy ** 2 + 1.0 / dz ** 2))


def material_coefficients(eps_r, sigma, dt):
    """Ca, Cb of the lossy E update for per-cell eps_r and sigma (arrays or scalars)."""
    eps = EPS0 * np.asarray(eps_r, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64) * dt / (2.0 * eps)
    ca = (1.0 - s) / (1.0 + s)
    cb = (dt / eps) / (1.0 + s)
    return ca, cb


def round_fp32(x):
    """fp32 storage emulation: round to binary32 (nearest even) and back."""
    return np.asarray(np.asarray(x, dtype=np.float64).astype(np.float32), dtype=np.float64)


def round_fp16_scaled(x, s: int):
    """fp16 storage emulation: round x*2^s to binary16 (nearest even), scale back.

    numpy's float64 -> float16 conversion rounds to nearest even and keeps
    subnormals; scaling by 2^s is exact in FP64.
    """
    scale = np.ldexp(1.0, s)
    return np.asarray(np.asarray(x * scale, dtype=np.float64).astype(np.float16),
                      dtype=np.float64) / scale


# ----------------------------------------------------------------------------
# Sources and probes
# ----------------------------------------------------------------------------

@dataclass
class Source:
    """Soft point source on one E sample: E[comp][i,j,k] += amp * w(t).

    kind "gauss_deriv": w(t) = -2 u exp(-u^2), u = (t - t0)/tau.
    kind "mod_gauss":   w(t) = sin(2 pi f0 (t - t0)) exp(-u^2).
    """
    comp: int
    i: int
    j: int
    k: int
    kind: str = "gauss_deriv"
    amp: float = 1.0
    t0: float = 0.0
    tau: float = 1.0
    f0: float = 0.0

    def waveform(self, t):
        u = (t - self.t0) / self.tau
        if self.kind == "gauss_deriv":
            return -2.0 * u * np.exp(-u * u)
        if self.kind == "mod_gauss":
            return np.sin(2.0 * np.pi * self.f0 * (t - self.t0)) * np.exp(-u * u)
        raise ValueError(f"unknown waveform {self.kind!r}")


@dataclass
class Probe:
    """Records component ``comp`` (0..5 = Ex..Hz) at (i, j, k) after every step."""
    comp: int
    i: int
    j: int
    k: int
    freqs: Optional[np.ndarray] = None


def dft_accumulate(acc, y, n, freqs, dt):
    """Running DFT: acc(f) + y exp(-i 2 pi f n dt) dt, phasor evaluated directly in FP64."""
    return acc + y * np.exp(-2j * np.pi * np.asarray(freqs, dtype=np.float64) * (n * dt)) * dt


# ----------------------------------------------------------------------------
# CPML profiles
# ----------------------------------------------------------------------------

@dataclass
class CpmlParams:
    cells: object = 0            # layer thickness L in cells: one int for all six faces,
                                 # or (Lx, Ly, Lz) per axis (0 = none on that axis)
    m: float = 3.0               # polynomial grading order
    sigma_max: Optional[float] = None   # None -> 0.8 (m+1)/(eta0 dw) per axis
    kappa_max: float = 1.0
    alpha_max: float = 0.0


def cpml_cells(p: CpmlParams):
    """Per-axis layer thickness (Lx, Ly, Lz)."""
    if isinstance(p.cells, (tuple, list)):
        return tuple(int(c) for c in p.cells)
    return (int(p.cells),) * 3


def cpml_profile(n: int, d: float, dt: float, p: CpmlParams, half: bool, L: int):
    """(b, a, 1/kappa) along one axis of n cells with a layer of L cells.

    Sample positions along the axis are integer (E side: the derivative of an
    E update sits where the E sample sits, 0..n) or half-integer (H side,
    0.5..n-0.5).  The normalised depth into the layer is
    x = max(L - p, p - (n - L), 0) / L, and
        sigma = sigma_max x^m,  kappa = 1 + (kappa_max - 1) x^m,
        alpha = alpha_max (1 - x),
        b = exp(-(sigma/kappa + alpha) dt/eps0),
        a = sigma (b - 1) / (kappa (sigma + kappa alpha))   (0 where sigma = 0).
    Outside the layer sigma = 0, so a = 0 and psi stays 0.
    """
    pos = np.arange(n, dtype=np.float64) + 0.5 if half else np.arange(n + 1, dtype=np.float64)
    if L <= 0:
        return np.ones_like(pos), np.zeros_like(pos), np.ones_like(pos)
    x = np.maximum(np.maximum(L - pos, pos - (n - L)), 0.0) / L
    smax = p.sigma_max if p.sigma_max is not None else 0.8 * (p.m + 1.0) / (ETA0 * d)
    sig = smax * x ** p.m
    kap = 1.0 + (p.kappa_max - 1.0) * x ** p.m
    alp = p.alpha_max * (1.0 - x)
    b = np.exp(-(sig / kap + alp) * dt / EPS0)
    denom = kap * (sig + kap * alp)
    a = np.where(sig > 0.0, sig * (b - 1.0) / np.where(denom > 0.0, denom, 1.0), 0.0)
    return b, a, 1.0 / kap


# ----------------------------------------------------------------------------
# The simulation
# ----------------------------------------------------------------------------

class Simulation:
    """One Yee grid advanced in FP64.

    Parameters
    ----------
    nx, ny, nz : number of cells; the box is [0, nx dx] x [0, ny dy] x [0, nz dz].
    eps_r, sigma : per-cell arrays of shape (nx, ny, nz) (or scalars).  The E
        sample [i,j,k] takes the cell (min(i,nx-1), min(j,ny-1), min(k,nz-1))
        (index-aligned staircase).
    pec : optional dict "Ex"/"Ey"/"Ez" -> bool array of that component's shape;
        True samples get Ca = Cb = 0.
    cpml : CpmlParams (cells = 0 for a plain PEC box).
    storage : "f64", "f16" (FP16-storage emulation with exponents fp16_exp
        for Ex, Ey, Ez, Hx, Hy, Hz) or "f32" (FP32-storage emulation).
    arith : "f64" or "f32" (the dtype of every array and operation; see the
        module documentation).
    """

    def __init__(self, nx, ny, nz, dx, dy=None, dz=None, courant=0.99,
                 eps_r=1.0, sigma=0.0, pec: Optional[Dict[str, np.ndarray]] = None,
                 cpml: Optional[CpmlParams] = None,
                 sources: Sequence[Source] = (), probes: Sequence[Probe] = (),
                 storage: str = "f64", fp16_exp=(0, 0, 0, 9, 9, 9), dt: Optional[float] = None,
                 arith: str = "f64"):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dx = float(dx)
        self.dy = float(dx if dy is None else dy)
        self.dz = float(dx if dz is None else dz)
        self.dt = float(time_step(self.dx, self.dy, self.dz, courant) if dt is None else dt)
        self.cpml = cpml if cpml is not None else CpmlParams()
        self.storage = storage
        if arith not in ("f64", "f32"):
            raise ValueError("arith must be 'f64' or 'f32'")
        self.arith = arith
        f = self.dtype = np.float32 if arith == "f32" else np.float64
        self.fp16_exp = tuple(int(s) for s in fp16_exp)
        self.sources: List[Source] = list(sources)
        self.probes: List[Probe] = list(probes)
        self.n = 0

        cells = (self.nx, self.ny, self.nz)
        eps_cell = np.broadcast_to(np.asarray(eps_r, dtype=np.float64), cells)
        sig_cell = np.broadcast_to(np.asarray(sigma, dtype=np.float64), cells)
        ca_cell, cb_cell = material_coefficients(eps_cell, sig_cell, self.dt)
        self.eps_cell = np.array(eps_cell)
        self.sig_cell = np.array(sig_cell)
        self.Ca: Dict[str, np.ndarray] = {}
        self.Cb: Dict[str, np.ndarray] = {}
        for c in E_COMPONENTS:
            shp = yee_shape(c, *cells)
            ii = np.minimum(np.arange(shp[0]), self.nx - 1)
            jj = np.minimum(np.arange(shp[1]), self.ny - 1)
            kk = np.minimum(np.arange(shp[2]), self.nz - 1)
            ca = ca_cell[np.ix_(ii, jj, kk)].copy()
            cb = cb_cell[np.ix_(ii, jj, kk)].copy()
            if pec is not None and c in pec:
                m = np.asarray(pec[c], dtype=bool)
                ca[m] = 0.0
                cb[m] = 0.0
            self.Ca[c], self.Cb[c] = ca.astype(f), cb.astype(f)

        # CPML profiles per axis: E side (integer positions), H side (half-integer).
        p = self.cpml
        self.pe, self.ph = {}, {}
        for ax, n, d, L in zip("xyz", (self.nx, self.ny, self.nz), (self.dx, self.dy, self.dz),
                               cpml_cells(p)):
            self.pe[ax] = tuple(v.astype(f) for v in cpml_profile(n, d, self.dt, p, half=False, L=L))
            self.ph[ax] = tuple(v.astype(f) for v in cpml_profile(n, d, self.dt, p, half=True, L=L))

        self.E = {c: np.zeros(yee_shape(c, *cells), dtype=f) for c in E_COMPONENTS}
        self.H = {c: np.zeros(yee_shape(c, *cells), dtype=f) for c in H_COMPONENTS}
        # psi arrays, named by (component, derivative axis); full size, zero
        # wherever a = 0 (outside the layer).
        nx_, ny_, nz_ = cells
        shapes = {
            "Hxy": (nx_ + 1, ny_, nz_), "Hxz": (nx_ + 1, ny_, nz_),
            "Hyz": (nx_, ny_ + 1, nz_), "Hyx": (nx_, ny_ + 1, nz_),
            "Hzx": (nx_, ny_, nz_ + 1), "Hzy": (nx_, ny_, nz_ + 1),
            "Exy": (nx_, ny_ - 1, nz_ - 1), "Exz": (nx_, ny_ - 1, nz_ - 1),
            "Eyz": (nx_ - 1, ny_, nz_ - 1), "Eyx": (nx_ - 1, ny_, nz_ - 1),
            "Ezx": (nx_ - 1, ny_ - 1, nz_), "Ezy": (nx_ - 1, ny_ - 1, nz_),
        }
        self.psi = {k: np.zeros(v, dtype=f) for k, v in shapes.items()}
        self.series: List[List[float]] = [[] for _ in self.probes]
        self.dft = [np.zeros(len(pr.freqs) if pr.freqs is not None else 0, dtype=np.complex128)
                    for pr in self.probes]

    # -- helpers --------------------------------------------------------------
    @staticmethod
    def _ax(v, axis):
        """Broadcast a 1-D profile along the given array axis (0, 1 or 2)."""
        shp = [1, 1, 1]
        shp[axis] = v.shape[0]
        return v.reshape(shp)

    def _store(self, comp_index, x):
        if self.storage == "f16":
            x = round_fp16_scaled(x, self.fp16_exp[comp_index])
        elif self.storage == "f32":
            x = round_fp32(x)
        return np.asarray(x, dtype=self.dtype)

    def set_fields(self, **arrays):
        """Set initial components (E^0 or H^{-1/2}); stored values are rounded
        like every other stored value in a storage-emulation mode."""
        for name, arr in arrays.items():
            idx = COMPONENTS.index(name)
            tgt = self.E if name in self.E else self.H
            a = np.array(arr, dtype=np.float64)
            assert a.shape == tgt[name].shape, (name, a.shape, tgt[name].shape)
            tgt[name] = self._store(idx, a)

    # -- one step -------------------------------------------------------------
    def step(self):
        """Advance (E^n, H^{n-1/2}) -> (E^{n+1}, H^{n+1/2})."""
        Ex, Ey, Ez = self.E["Ex"], self.E["Ey"], self.E["Ez"]
        Hx, Hy, Hz = self.H["Hx"], self.H["Hy"], self.H["Hz"]
        dx, dy, dz, dt = self.dx, self.dy, self.dz, self.dt
        P, A = self.psi, self._ax
        bhx, ahx, khx = self.ph["x"]
        bhy, ahy, khy = self.ph["y"]
        bhz, ahz, khz = self.ph["z"]
        bex, aex, kex = self.pe["x"]
        bey, aey, key = self.pe["y"]
        bez, aez, kez = self.pe["z"]
        dt_mu = dt / MU0

        # ---- H half step: H^{n+1/2} = H^{n-1/2} - (dt/mu0) curl E^n ----
        dyEz = (Ez[:, 1:, :] - Ez[:, :-1, :]) / dy
        dzEy = (Ey[:, :, 1:] - Ey[:, :, :-1]) / dz
        P["Hxy"] = A(bhy, 1) * P["Hxy"] + A(ahy, 1) * dyEz
        P["Hxz"] = A(bhz, 2) * P["Hxz"] + A(ahz, 2) * dzEy
        Hx_new = Hx - dt_mu * ((A(khy, 1) * dyEz + P["Hxy"]) - (A(khz, 2) * dzEy + P["Hxz"]))

        dzEx = (Ex[:, :, 1:] - Ex[:, :, :-1]) / dz
        dxEz = (Ez[1:, :, :] - Ez[:-1, :, :]) / dx
        P["Hyz"] = A(bhz, 2) * P["Hyz"] + A(ahz, 2) * dzEx
        P["Hyx"] = A(bhx, 0) * P["Hyx"] + A(ahx, 0) * dxEz
        Hy_new = Hy - dt_mu * ((A(khz, 2) * dzEx + P["Hyz"]) - (A(khx, 0) * dxEz + P["Hyx"]))

        dxEy = (Ey[1:, :, :] - Ey[:-1, :, :]) / dx
        dyEx = (Ex[:, 1:, :] - Ex[:, :-1, :]) / dy
        P["Hzx"] = A(bhx, 0) * P["Hzx"] + A(ahx, 0) * dxEy
        P["Hzy"] = A(bhy, 1) * P["Hzy"] + A(ahy, 1) * dyEx
        Hz_new = Hz - dt_mu * ((A(khx, 0) * dxEy + P["Hzx"]) - (A(khy, 1) * dyEx + P["Hzy"]))

        Hx = self.H["Hx"] = self._store(3, Hx_new)
        Hy = self.H["Hy"] = self._store(4, Hy_new)
        Hz = self.H["Hz"] = self._store(5, Hz_new)

        # ---- E half step on interior (non-wall) samples ----
        nx, ny, nz = self.nx, self.ny, self.nz
        # Ex[:, 1:ny, 1:nz]
        dyHz = (Hz[:, 1:ny, 1:nz] - Hz[:, 0:ny - 1, 1:nz]) / dy
        dzHy = (Hy[:, 1:ny, 1:nz] - Hy[:, 1:ny, 0:nz - 1]) / dz
        P["Exy"] = A(bey[1:ny], 1) * P["Exy"] + A(aey[1:ny], 1) * dyHz
        P["Exz"] = A(bez[1:nz], 2) * P["Exz"] + A(aez[1:nz], 2) * dzHy
        rx = (A(key[1:ny], 1) * dyHz + P["Exy"]) - (A(kez[1:nz], 2) * dzHy + P["Exz"])
        s = (slice(None), slice(1, ny), slice(1, nz))
        Ex_new = Ex.copy()
        Ex_new[s] = self.Ca["Ex"][s] * Ex[s] + self.Cb["Ex"][s] * rx

        # Ey[1:nx, :, 1:nz]
        dzHx = (Hx[1:nx, :, 1:nz] - Hx[1:nx, :, 0:nz - 1]) / dz
        dxHz = (Hz[1:nx, :, 1:nz] - Hz[0:nx - 1, :, 1:nz]) / dx
        P["Eyz"] = A(bez[1:nz], 2) * P["Eyz"] + A(aez[1:nz], 2) * dzHx
        P["Eyx"] = A(bex[1:nx], 0) * P["Eyx"] + A(aex[1:nx], 0) * dxHz
        ry = (A(kez[1:nz], 2) * dzHx + P["Eyz"]) - (A(kex[1:nx], 0) * dxHz + P["Eyx"])
        s = (slice(1, nx), slice(None), slice(1, nz))
        Ey_new = Ey.copy()
        Ey_new[s] = self.Ca["Ey"][s] * Ey[s] + self.Cb["Ey"][s] * ry

        # Ez[1:nx, 1:ny, :]
        dxHy = (Hy[1:nx, 1:ny, :] - Hy[0:nx - 1, 1:ny, :]) / dx
        dyHx = (Hx[1:nx, 1:ny, :] - Hx[1:nx, 0:ny - 1, :]) / dy
        P["Ezx"] = A(bex[1:nx], 0) * P["Ezx"] + A(aex[1:nx], 0) * dxHy
        P["Ezy"] = A(bey[1:ny], 1) * P["Ezy"] + A(aey[1:ny], 1) * dyHx
        rz = (A(kex[1:nx], 0) * dxHy + P["Ezx"]) - (A(key[1:ny], 1) * dyHx + P["Ezy"])
        s = (slice(1, nx), slice(1, ny), slice(None))
        Ez_new = Ez.copy()
        Ez_new[s] = self.Ca["Ez"][s] * Ez[s] + self.Cb["Ez"][s] * rz

        # ---- soft sources at t = (n+1) dt ----
        # the bracketed curl terms of this E update (interior samples), kept for
        # the adjoint's gradient: E^{n+1} = Ca E^n + Cb R^n
        self.last_r = {"Ex": rx, "Ey": ry, "Ez": rz}
        new = {"Ex": Ex_new, "Ey": Ey_new, "Ez": Ez_new}
        t = (self.n + 1) * dt
        for src in self.sources:
            new[E_COMPONENTS[src.comp]][src.i, src.j, src.k] += src.amp * src.waveform(t)
        for ci, c in enumerate(E_COMPONENTS):
            self.E[c] = self._store(ci, new[c])

        self.n += 1
        # ---- probes and running DFT ----
        for p_i, pr in enumerate(self.probes):
            y = self.component(pr.comp)[pr.i, pr.j, pr.k]
            self.series[p_i].append(float(y))
            if pr.freqs is not None and len(pr.freqs):
                self.dft[p_i] = dft_accumulate(self.dft[p_i], y, self.n, pr.freqs, dt)

    def run(self, nsteps: int):
        for _ in range(int(nsteps)):
            self.step()
        return self

    # -- accessors ------------------------------------------------------------
    def component(self, comp):
        name = COMPONENTS[comp] if isinstance(comp, (int, np.integer)) else comp
        return self.E[name] if name in self.E else self.H[name]

    def series_array(self) -> np.ndarray:
        """Probe series as an array [n_steps, n_probes]."""
        if not self.probes:
            return np.zeros((self.n, 0))
        return np.array(self.series, dtype=np.float64).T

    def energy(self, e_n: Dict[str, np.ndarray], h_prev: Dict[str, np.ndarray],
               h_next: Dict[str, np.ndarray]) -> float:
        """Discrete Yee energy W^n = 1/2 sum eps |E^n|^2 dV + 1/2 sum mu0 H^{n-1/2}.H^{n+1/2} dV.

        For sigma = 0 this is invariant under the leapfrog (the E and H curl
        operators are transposes of each other), so it is the conserved
        quantity of a closed lossless PEC box.  Each E sample carries its
        cell's eps (index-aligned staircase).
        """
        dv = self.dx * self.dy * self.dz
        w = 0.0
        for c in E_COMPONENTS:
            shp = e_n[c].shape
            ii = np.minimum(np.arange(shp[0]), self.nx - 1)
            jj = np.minimum(np.arange(shp[1]), self.ny - 1)
            kk = np.minimum(np.arange(shp[2]), self.nz - 1)
            eps = EPS0 * self.eps_cell[np.ix_(ii, jj, kk)]
            w += 0.5 * float(np.sum(eps * e_n[c] ** 2)) * dv
        for c in H_COMPONENTS:
            w += 0.5 * MU0 * float(np.sum(h_prev[c] * h_next[c])) * dv
        return w
