"""FP64 discrete adjoint of the Yee step (reverse-mode derivative).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Objective: J = sum over steps n = 1..N and probe samples p of (F_p^n)^2, where
F_p^n is the probed component (any of Ex..Hz; a bare (i, j, k) means Ez) in
the state after step n (E^n and H^{n-1/2}).
Gradient: dJ/d eps_r for every cell, with eps_r entering through the lossy
update coefficients Ca, Cb of the cell's three E samples (index-aligned
staircase).  The paper defines no solver and no adjoint; this is reverse-mode
differentiation of the textbook scheme in :mod:`oracle.yee`, written as the
transpose of each sub-map of one step, applied in reverse order:

  forward step n:  (1) psi_H <- b psi_H + a D E        (2) H <- H - (dt/mu0)(K C_e E + S psi_H)
                   (3) psi_E <- b psi_E + a D H        (4) E <- Ca E + Cb (K C_h H + S psi_E)
                   (5) E <- E + source (state independent)
                   (6) J <- J + sum_p F[p]^2
  reverse step n:  (6^T) F_bar[p] += 2 F[p] (E^{n+1} or H^{n+1/2})
                   (4^T) R_bar = Cb E_bar; psi_E_bar += S^T R_bar; H_bar += C_h^T (K R_bar) + D^T (a psi_E_bar);
                         grad += E_bar (dCa/deps E^n + dCb/deps R^n); E_bar <- Ca E_bar; psi_E_bar <- b psi_E_bar
                   (2^T, 1^T) psi_H_bar += -(dt/mu0) S^T H_bar; E_bar += C_e^T(-(dt/mu0) K H_bar) + D^T (a psi_H_bar);
                         psi_H_bar <- b psi_H_bar
where R^n is the bracketed curl term of the E update at step n.  The forward
states are regenerated segment by segment from checkpoints taken every K steps.
"""
from __future__ import annotations

import copy
from typing import Callable, List, Sequence, Tuple

import numpy as np

from .yee import EPS0, MU0, Simulation

COMPONENTS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")


def _probe_list(probes):
    """(comp, i, j, k) tuples with comp in 0..5; a 3-tuple (i, j, k) is an Ez probe."""
    out = []
    for p in probes:
        out.append((2,) + tuple(p) if len(p) == 3 else tuple(p))
    return out


def _probe_value(E, H, p):
    c, i, j, k = p
    return float((E if c < 3 else H)[COMPONENTS[c]][i, j, k])


def coefficient_derivatives(eps_r, sigma, dt):
    """dCa/d eps_r and dCb/d eps_r of the semi-implicit lossy update.

    With s = sigma dt/(2 eps0 eps_r): Ca = (1-s)/(1+s), Cb = (dt/(eps0 eps_r))/(1+s),
    ds/d eps_r = -s/eps_r, so dCa/d eps_r = 2 s/(eps_r (1+s)^2) and
    dCb/d eps_r = -Cb/(eps_r (1+s))."""
    eps_r = np.asarray(eps_r, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64) * dt / (2.0 * EPS0 * eps_r)
    cb = (dt / (EPS0 * eps_r)) / (1.0 + s)
    return 2.0 * s / (eps_r * (1.0 + s) ** 2), -cb / (eps_r * (1.0 + s))


def _state(sim: Simulation):
    return (copy.deepcopy(sim.E), copy.deepcopy(sim.H), copy.deepcopy(sim.psi), sim.n,
            [list(s) for s in sim.series], copy.deepcopy(sim.dft))


def _restore(sim: Simulation, st):
    sim.E, sim.H, sim.psi = copy.deepcopy(st[0]), copy.deepcopy(st[1]), copy.deepcopy(st[2])
    sim.n = st[3]
    sim.series = [list(s) for s in st[4]]
    sim.dft = copy.deepcopy(st[5])


class Adjoint:
    """Adjoint state of one simulation and the reverse of one step."""

    def __init__(self, sim: Simulation, probes: Sequence[Tuple[int, int, int]]):
        self.sim = sim
        self.probes = _probe_list(probes)
        self.aE = {c: np.zeros_like(v) for c, v in sim.E.items()}
        self.aH = {c: np.zeros_like(v) for c, v in sim.H.items()}
        self.ap = {c: np.zeros_like(v) for c, v in sim.psi.items()}
        self.grad = np.zeros((sim.nx, sim.ny, sim.nz))
        dca, dcb = coefficient_derivatives(sim.eps_cell, sim.sig_cell, sim.dt)
        # per-sample derivatives; masked (PEC) samples do not depend on eps_r
        self.dCa, self.dCb = {}, {}
        for c in ("Ex", "Ey", "Ez"):
            shp = sim.E[c].shape
            ii = np.minimum(np.arange(shp[0]), sim.nx - 1)
            jj = np.minimum(np.arange(shp[1]), sim.ny - 1)
            kk = np.minimum(np.arange(shp[2]), sim.nz - 1)
            live = sim.Cb[c] != 0.0
            self.dCa[c] = np.where(live, dca[np.ix_(ii, jj, kk)], 0.0)
            self.dCb[c] = np.where(live, dcb[np.ix_(ii, jj, kk)], 0.0)

    def reverse_step(self, E_n, R_n, E_np1, H_np1=None, objective=True, gradient=True):
        """Map the adjoint of the state after a step to the adjoint before it.

        E_n: E before the step; R_n: its bracketed curl terms; E_np1, H_np1: the
        state after the step (H_np1 is needed only for H probes)."""
        sim = self.sim
        aE, aH, ap = self.aE, self.aH, self.ap
        nx, ny, nz = sim.nx, sim.ny, sim.nz
        dx, dy, dz = sim.dx, sim.dy, sim.dz
        A = sim._ax
        bex, aex, kex = sim.pe["x"]
        bey, aey, key = sim.pe["y"]
        bez, aez, kez = sim.pe["z"]
        bhx, ahx, khx = sim.ph["x"]
        bhy, ahy, khy = sim.ph["y"]
        bhz, ahz, khz = sim.ph["z"]

        # (6^T) objective: d/dF of sum_p F[p]^2 on the state after the step
        if objective:
            for p in self.probes:
                c, i, j, k = p
                tgt = aE if c < 3 else aH
                tgt[COMPONENTS[c]][i, j, k] += 2.0 * _probe_value(E_np1, H_np1, p)

        # (4^T, 3^T) E update, per component, on its interior samples
        def e_transpose(c, s, cells, terms):
            ebar = aE[c][s]
            rbar = sim.Cb[c][s] * ebar
            if gradient:
                self.grad[cells] += ebar * (self.dCa[c][s] * E_n[c][s] + self.dCb[c][s] * R_n[c])
            for (pname, sign, kap, bprof, aprof, hname, axis, d) in terms:
                ap[pname] += sign * rbar
                dbar = sign * kap * rbar + aprof * ap[pname]
                ap[pname] *= bprof
                # transpose of the backward difference (H[m] - H[m-1])/d along `axis`
                hi = list(s)
                lo = list(s)
                hi[axis] = s[axis]
                lo[axis] = slice(s[axis].start - 1, s[axis].stop - 1)
                aH[hname][tuple(hi)] += dbar / d
                aH[hname][tuple(lo)] -= dbar / d
            aE[c][s] = sim.Ca[c][s] * ebar

        sx = (slice(0, nx), slice(1, ny), slice(1, nz))
        e_transpose("Ex", sx, (slice(None), slice(1, ny), slice(1, nz)), [
            ("Exy", +1.0, A(key[1:ny], 1), A(bey[1:ny], 1), A(aey[1:ny], 1), "Hz", 1, dy),
            ("Exz", -1.0, A(kez[1:nz], 2), A(bez[1:nz], 2), A(aez[1:nz], 2), "Hy", 2, dz)])
        sy = (slice(1, nx), slice(0, ny), slice(1, nz))
        e_transpose("Ey", sy, (slice(1, nx), slice(None), slice(1, nz)), [
            ("Eyz", +1.0, A(kez[1:nz], 2), A(bez[1:nz], 2), A(aez[1:nz], 2), "Hx", 2, dz),
            ("Eyx", -1.0, A(kex[1:nx], 0), A(bex[1:nx], 0), A(aex[1:nx], 0), "Hz", 0, dx)])
        sz = (slice(1, nx), slice(1, ny), slice(0, nz))
        e_transpose("Ez", sz, (slice(1, nx), slice(1, ny), slice(None)), [
            ("Ezx", +1.0, A(kex[1:nx], 0), A(bex[1:nx], 0), A(aex[1:nx], 0), "Hy", 0, dx),
            ("Ezy", -1.0, A(key[1:ny], 1), A(bey[1:ny], 1), A(aey[1:ny], 1), "Hx", 1, dy)])

        # (2^T, 1^T) H update: H' = H - (dt/mu0) [(k1 d1 + psi1) - (k2 d2 + psi2)]
        mu = sim.dt / MU0

        def h_transpose(hname, terms):
            hbar = aH[hname]
            for (pname, sign, kap, bprof, aprof, ename, axis, d) in terms:
                ap[pname] += -mu * sign * hbar
                dbar = -mu * sign * kap * hbar + aprof * ap[pname]
                ap[pname] *= bprof
                # transpose of the forward difference (E[m+1] - E[m])/d along `axis`
                hi = [slice(None)] * 3
                lo = [slice(None)] * 3
                hi[axis] = slice(1, None)
                lo[axis] = slice(0, -1)
                aE[ename][tuple(hi)] += dbar / d
                aE[ename][tuple(lo)] -= dbar / d

        h_transpose("Hx", [("Hxy", +1.0, A(khy, 1), A(bhy, 1), A(ahy, 1), "Ez", 1, dy),
                           ("Hxz", -1.0, A(khz, 2), A(bhz, 2), A(ahz, 2), "Ey", 2, dz)])
        h_transpose("Hy", [("Hyz", +1.0, A(khz, 2), A(bhz, 2), A(ahz, 2), "Ex", 2, dz),
                           ("Hyx", -1.0, A(khx, 0), A(bhx, 0), A(ahx, 0), "Ez", 0, dx)])
        h_transpose("Hz", [("Hzx", +1.0, A(khx, 0), A(bhx, 0), A(ahx, 0), "Ey", 0, dx),
                           ("Hzy", -1.0, A(khy, 1), A(bhy, 1), A(ahy, 1), "Ex", 1, dy)])


def objective(make_sim: Callable[[], Simulation], nsteps: int, probes) -> float:
    """J = sum_{n=1}^{N} sum_p (F_p^n)^2 of a fresh simulation."""
    probes = _probe_list(probes)
    sim = make_sim()
    j = 0.0
    for _ in range(nsteps):
        sim.step()
        for p in probes:
            j += _probe_value(sim.E, sim.H, p) ** 2
    return j


def gradient(make_sim: Callable[[], Simulation], nsteps: int, probes, checkpoint_every: int = 64):
    """(J, dJ/d eps_r per cell) by the discrete adjoint with checkpoint-recompute."""
    probes = _probe_list(probes)
    sim = make_sim()
    ckpts: List = []
    j = 0.0
    for n in range(nsteps):
        if n % checkpoint_every == 0:
            ckpts.append(_state(sim))
        sim.step()
        for p in probes:
            j += _probe_value(sim.E, sim.H, p) ** 2
    adj = Adjoint(sim, probes)
    for seg in reversed(range(len(ckpts))):
        n0 = seg * checkpoint_every
        n1 = min(nsteps, n0 + checkpoint_every)
        _restore(sim, ckpts[seg])
        hist_e, hist_h, hist_r = [copy.deepcopy(sim.E)], [None], []
        for _ in range(n0, n1):
            sim.step()
            hist_e.append(copy.deepcopy(sim.E))
            hist_h.append(copy.deepcopy(sim.H))
            hist_r.append(copy.deepcopy(sim.last_r))
        for m in reversed(range(n1 - n0)):
            adj.reverse_step(hist_e[m], hist_r[m], hist_e[m + 1], hist_h[m + 1])
    return j, adj.grad
