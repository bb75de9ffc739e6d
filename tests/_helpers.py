"""Shared test plumbing: build the oracle and the HIP solver from one workload."""
import numpy as np

from oracle.yee import CpmlParams, Probe, Simulation, Source


def oracle_from_workload(wl, initial=None, storage=None, dt=None, arith="f64"):
    eps, sig = wl.cell_materials()
    cp = CpmlParams(cells=tuple(wl.cpml_cells), m=wl.cpml_m, sigma_max=wl.cpml_sigma_max,
                    kappa_max=wl.cpml_kappa_max, alpha_max=wl.cpml_alpha_max)
    sim = Simulation(wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, courant=wl.courant, eps_r=eps, sigma=sig,
                     pec=wl.pec_component_masks(), cpml=cp,
                     storage=storage or ("f16" if wl.precision == "f16" else "f64"),
                     fp16_exp=wl.fp16_exp, dt=dt, arith=arith)
    srcs = []
    for s in wl.sources:
        t0, tau = s.times(sim.dt)
        srcs.append(Source(s.comp, s.i, s.j, s.k, s.kind, s.amp, t0, tau, s.f0))
    sim.sources = srcs
    sim.probes = [Probe(c, i, j, k, np.asarray(wl.freqs) if len(wl.freqs) else None) for (c, i, j, k) in wl.probes]
    sim.series = [[] for _ in sim.probes]
    sim.dft = [np.zeros(len(wl.freqs), complex) for _ in sim.probes]
    if initial is not None:
        full = {}
        for name, arr in initial.items():
            tgt = sim.component(name)
            a = np.zeros(tgt.shape)
            a[:wl.nx, :wl.ny, :wl.nz] = arr
            full[name] = a
        sim.set_fields(**full)
    return sim


def stored(sim, comp):
    """Oracle component restricted to the stored range (i < nx, j < ny, k < nz)."""
    return sim.component(comp)[:sim.nx, :sim.ny, :sim.nz]


def rel_l2(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((x - ref).ravel())
    if den == 0.0:
        return 0.0 if num == 0.0 else np.inf
    return num / den
