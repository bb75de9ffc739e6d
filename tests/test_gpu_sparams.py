"""Two-run S-parameters from the HIP solver's FP64 running DFTs (FP32 fields)
through the library (yee_sparams), against the same extraction on the FP64
oracle's runs, on the PEC-waveguide workloads (reference, PEC short,
dielectric slab).  Gate: |S_gpu - S_oracle| <= 1e-4 (the FP32 solve moves
the probe DFTs by about 1e-5 relative); the short's phase pin holds on the
GPU result too."""
import sys

import numpy as np
import pytest

from _helpers import oracle_from_workload
from oracle import sparams as SP
from paper_2305_14176_amd import workloads as W

pytestmark = pytest.mark.gpu
PORTS = [([0], [1.0]), ([1], [1.0])]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(600)
def test_gpu_sparams_match_oracle():
    import torch
    assert torch.cuda.is_available()
    from paper_2305_14176_amd import sparams as L
    from paper_2305_14176_amd.solver import YeeSolver
    from test_oracle_sparams import discrete_beta
    gpu, ora = {}, {}
    for kind in ("ref", "short", "slab"):
        wl = W.waveguide_ports(kind, precision="f32")
        _say(f"[gpu] sparams waveguide {kind}: {wl.nx}x{wl.ny}x{wl.nz}, {wl.steps} steps")
        s = YeeSolver(wl, device="cuda:0")
        s.step(wl.steps)
        gpu[kind] = s.dft()
        s.close()
        sim = oracle_from_workload(W.waveguide_ports(kind, precision="f64"))
        sim.run(wl.steps)
        ora[kind] = np.array(sim.dft)
        odt = sim.dt
    pp, pw = [p for p, _ in PORTS], [w for _, w in PORTS]
    for kind in ("short", "slab"):
        _, _, s_gpu = L.sparams(gpu["ref"], gpu[kind], PORTS)
        s_ora = SP.two_run(SP.port_voltages(ora["ref"], pp, pw), SP.port_voltages(ora[kind], pp, pw))
        err = np.abs(s_gpu - s_ora).max()
        _say(f"[gpu]   {kind}: max |S_gpu - S_oracle| = {err:.2e}")
        assert err <= 1e-4, (kind, err)
    wl = W.waveguide_ports("short")
    _, _, s = L.sparams(gpu["ref"], gpu["short"], PORTS)
    pred = np.exp(-2j * discrete_beta(wl, odt) * (90 - 60.5) * wl.dz)
    assert np.abs(s[0] - pred).max() <= 0.03
    assert np.all(s[1] == 0)
