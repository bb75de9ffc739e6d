"""Pins of the port-voltage and two-run S-parameter oracle (oracle/sparams.py)
on FP64 FDTD runs of a PEC waveguide (workloads.waveguide_ports), and the
library's host implementation (yee_sparams) against the oracle.

Physical pins (independent of the S formulas themselves):
  * PEC short: tangential E vanishes on the short's plane z_s, so the discrete
    TM11 standing wave has Ez proportional to cos(beta (z - z_s)) on the
    half-integer Ez nodes, and S_11 at the probe (k = 60, z = 60.5 dz) is
    exp(-2 i beta (z_s - z_p)) with the Yee grid's own propagation constant
    (2/dz)^2 sin^2(beta dz/2) = (2/(c dt))^2 sin^2(w dt/2) - 2 (2/d)^2 sin^2(pi d/(2a)).
    Behind the short nothing arrives: S_21 = 0 exactly.
  * Lossless slab between the ports (same guide, same mode on both sides):
    |S_11|^2 + |S_21|^2 = 1.
  * Identical runs: S_11 = 0 exactly and S_21 = 1 to the last bit of a
    complex division.
The 0.03 bounds cover the band edges, where TM11 energy near cutoff (zero group
velocity) still rings when the run ends; mid-band the errors are a few 1e-3.
A half-cell slip of the reference plane would cost 0.4 rad, the continuum
propagation constant more than 0.1 rad.
"""
import os

import numpy as np
import pytest

from _helpers import oracle_from_workload
from oracle import sparams as SP
from paper_2305_14176_amd import workloads as W

C0 = 299792458.0
PORTS = [([0], [1.0]), ([1], [1.0])]
TOL = 0.03


def _ports(ports):
    return [p for p, _ in ports], [w for _, w in ports]


@pytest.fixture(scope="module")
def runs():
    out = {}
    for kind in ("ref", "short", "slab"):
        wl = W.waveguide_ports(kind, precision="f64")
        sim = oracle_from_workload(wl)
        sim.run(wl.steps)
        out[kind] = (wl, sim.dt, np.array(sim.dft))
    return out


def _s(runs, kind, ref="ref"):
    pp, pw = _ports(PORTS)
    return SP.two_run(SP.port_voltages(runs[ref][2], pp, pw), SP.port_voltages(runs[kind][2], pp, pw))


def discrete_beta(wl, dt):
    f = np.asarray(wl.freqs)
    d = wl.dx
    a = wl.nx * wl.dx
    rhs = (2 / (C0 * dt)) ** 2 * np.sin(np.pi * f * dt) ** 2 - 2 * (2 / d) ** 2 * np.sin(np.pi * d / (2 * a)) ** 2
    assert np.all(rhs > 0), "every frequency must propagate"
    return 2 / wl.dz * np.arcsin(np.sqrt(rhs) * wl.dz / 2)


def test_short_reflects_with_the_discrete_phase(runs):
    wl, dt, _ = runs["short"]
    s = _s(runs, "short")
    pred = np.exp(-2j * discrete_beta(wl, dt) * (90 - 60.5) * wl.dz)
    err = np.abs(s[0] - pred)
    assert err.max() <= TOL, err
    assert np.all(s[1] == 0)


def test_lossless_slab_conserves_power(runs):
    s = _s(runs, "slab")
    p = np.abs(s[0]) ** 2 + np.abs(s[1]) ** 2
    assert np.abs(p - 1).max() <= TOL, p
    assert np.abs(s[0]).max() > 0.2 and np.abs(s[1]).min() < 0.95   # the slab does reflect


def test_identical_runs_give_no_reflection(runs):
    s = _s(runs, "ref", ref="ref")
    assert np.all(s[0] == 0)
    assert np.abs(s[1] - 1).max() <= 1e-15      # complex division v / v: within an ulp of 1


LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2305_14176_amd", "libyee.so")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libyee.so not built")
def test_library_matches_oracle(runs):
    from paper_2305_14176_amd import sparams as L
    for kind in ("short", "slab"):
        vr, vd, s = L.sparams(runs["ref"][2], runs[kind][2], PORTS)
        ref = _s(runs, kind)
        assert np.abs(s - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    rng = np.random.default_rng(11)
    a = rng.normal(size=(6, 5)) + 1j * rng.normal(size=(6, 5))
    b = rng.normal(size=(6, 5)) + 1j * rng.normal(size=(6, 5))
    ports = [([0, 2, 5], [0.5, 0.25, -1.0]), ([4], [2.0]), ([1, 3], [1.0, 1.0])]
    pp, pw = [p for p, _ in ports], [w for _, w in ports]
    vr, vd, s = L.sparams(a, b, ports)
    np.testing.assert_allclose(vr, SP.port_voltages(a, pp, pw), rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(vd, SP.port_voltages(b, pp, pw), rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(s, SP.two_run(SP.port_voltages(a, pp, pw), SP.port_voltages(b, pp, pw)),
                               rtol=1e-13, atol=1e-13)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libyee.so not built")
def test_library_rejects_bad_ports():
    from paper_2305_14176_amd import _lib
    from paper_2305_14176_amd import sparams as L
    a = np.ones((3, 4), complex)
    for ports in ([([3], [1.0])], [([-1], [1.0])], [([], [])], []):
        with pytest.raises(_lib.YeeError):
            L.sparams(a, a, ports)
    with pytest.raises(ValueError):
        L.sparams(a, a, [([0, 1], [1.0])])
