"""Pins of the oracle's discrete adjoint.

* The reverse step is the exact transpose of the forward step: for random
  states x and adjoints l, <l, L x> = <L^T l, x> (L = one source-free step,
  CPML with kappa and alpha, lossy materials and a PEC plane included).
* The gradient equals central finite differences of the objective (FP64,
  h = 1e-3 on eps_r), on cells inside, at the edge of and outside the CPML,
  for Ez probes and for probes of every E and H component.
* The coefficient derivatives match finite differences of Ca, Cb.
"""
import numpy as np
import pytest

from oracle.adjoint import Adjoint, coefficient_derivatives, gradient, objective
from oracle.yee import CpmlParams, Simulation, Source, material_coefficients


def _sim(eps, sig, pec_k=None, sources=True):
    nx, ny, nz = eps.shape
    pec = None
    if pec_k is not None:
        pec = {"Ex": np.zeros((nx, ny + 1, nz + 1), bool), "Ey": np.zeros((nx + 1, ny, nz + 1), bool)}
        pec["Ex"][2:5, 3:5, pec_k] = True
        pec["Ey"][3:6, 2:4, pec_k] = True
    sim = Simulation(nx, ny, nz, 1e-3, 1.1e-3, 0.9e-3, eps_r=eps, sigma=sig, pec=pec,
                     cpml=CpmlParams(cells=(2, 2, 2), kappa_max=1.6, alpha_max=0.03))
    if sources:
        dt = sim.dt
        sim.sources = [Source(2, 4, 4, 3, "mod_gauss", 1.0, 8 * dt, 3 * dt, 40e9)]
    return sim


def _materials(seed, shape=(9, 8, 7)):
    rng = np.random.default_rng(seed)
    return rng.uniform(1.0, 5.0, shape), rng.uniform(0.0, 0.5, shape)


def test_coefficient_derivatives_match_finite_differences():
    rng = np.random.default_rng(0)
    eps = rng.uniform(1, 10, 50)
    sig = rng.uniform(0, 3, 50)
    dt = 1e-12
    h = 1e-6
    dca, dcb = coefficient_derivatives(eps, sig, dt)
    ca_p, cb_p = material_coefficients(eps + h, sig, dt)
    ca_m, cb_m = material_coefficients(eps - h, sig, dt)
    np.testing.assert_allclose(dca, (ca_p - ca_m) / (2 * h), rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(dcb, (cb_p - cb_m) / (2 * h), rtol=1e-6, atol=0)


def _random_state(sim, rng):
    for d in (sim.E, sim.H, sim.psi):
        for c in d:
            d[c] = rng.standard_normal(d[c].shape) * (1.0 if c.startswith("E") else 1e-3)


def test_reverse_step_is_transpose_of_forward_step():
    rng = np.random.default_rng(1)
    eps, sig = _materials(2)
    sim = _sim(eps, sig, pec_k=3, sources=False)
    _random_state(sim, rng)
    x = {("E", c): v.copy() for c, v in sim.E.items()}
    x.update({("H", c): v.copy() for c, v in sim.H.items()})
    x.update({("P", c): v.copy() for c, v in sim.psi.items()})
    e_n = {c: v.copy() for c, v in sim.E.items()}
    sim.step()
    lx = {("E", c): v for c, v in sim.E.items()}
    lx.update({("H", c): v for c, v in sim.H.items()})
    lx.update({("P", c): v for c, v in sim.psi.items()})
    adj = Adjoint(sim, probes=[])
    lam = {}
    for key in x:
        lam[key] = rng.standard_normal(x[key].shape)
    for c in adj.aE:
        adj.aE[c] = lam[("E", c)].copy()
    for c in adj.aH:
        adj.aH[c] = lam[("H", c)].copy()
    for c in adj.ap:
        adj.ap[c] = lam[("P", c)].copy()
    adj.reverse_step(e_n, sim.last_r, sim.E, objective=False, gradient=False)
    ltl = {("E", c): v for c, v in adj.aE.items()}
    ltl.update({("H", c): v for c, v in adj.aH.items()})
    ltl.update({("P", c): v for c, v in adj.ap.items()})
    lhs = sum(float(np.sum(lam[k] * lx[k])) for k in x)
    rhs = sum(float(np.sum(ltl[k] * x[k])) for k in x)
    scale = sum(float(np.sum(np.abs(lam[k] * lx[k]))) for k in x)
    assert abs(lhs - rhs) <= 1e-13 * scale, (lhs, rhs)


@pytest.mark.parametrize("ckpt,probes", [
    (64, [(6, 5, 4), (2, 6, 2)]),
    (7, [(6, 5, 4), (2, 6, 2)]),
    # Ex and Ey probes, one sample probed twice
    (16, [(0, 5, 4, 3), (1, 4, 4, 4), (1, 4, 4, 4)]),
    # H probes only (H is ~1/377 of E: mixed with E probes its terms would vanish in J)
    (16, [(4, 3, 5, 2), (5, 6, 2, 4), (3, 2, 3, 5), (3, 2, 3, 5)]),
])
def test_gradient_matches_central_differences(ckpt, probes):
    eps, sig = _materials(3)
    nsteps = 45

    def make(e):
        return lambda: _sim(e, sig, pec_k=4)

    j, g = gradient(make(eps), nsteps, probes, checkpoint_every=ckpt)
    assert abs(j - objective(make(eps), nsteps, probes)) <= 1e-14 * j
    h = 1e-3
    cells = [(4, 4, 3), (5, 4, 4), (1, 1, 1), (3, 6, 5), (7, 2, 2), (4, 3, 4)]
    gmax = np.abs(g).max()
    assert gmax > 0
    for c in cells:
        ep, em = eps.copy(), eps.copy()
        ep[c] += h
        em[c] -= h
        fd = (objective(make(ep), nsteps, probes) - objective(make(em), nsteps, probes)) / (2 * h)
        assert abs(fd - g[c]) <= 1e-5 * gmax + 1e-5 * abs(g[c]), (c, fd, g[c])
