"""GPU parity: the HIP step (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances (relative L2 per output: each probe series, each probe's DFT
vector, each final field component):
  * FP64 mode  : 1e-12  (only rounding order and FMA contraction differ);
  * FP32 mode  : 1e-5   against the FP64 oracle (after the pulse has left a
                  CPML grid: three times the oracle's own FP32-storage drift);
  * FP16 storage: 1e-3  against the oracle emulating FP16 storage, over runs
                  short enough that the two take the same rounding decisions
                  almost everywhere (the long FP16 run is gated in
                  test_gpu_golden.py against the size of the storage error).
"""
import sys

import numpy as np
import pytest

from paper_2305_14176_amd import workloads as W
from _helpers import oracle_from_workload, rel_l2, stored

pytestmark = pytest.mark.gpu

COMPS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")
TOL = {"f64": 1e-12, "f32": 1e-5, "f16": 1e-3}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def solver_cls():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_14176_amd.solver import YeeSolver
    return YeeSolver


def _run_both(solver_cls, wl, steps, init_seed=None, storage=None, series_len=None, **kw):
    init = W.random_initial_fields(wl, init_seed) if init_seed is not None else None
    _say(f"[gpu] {wl.name} prec={wl.precision} steps={steps} init={init_seed} kw={kw}")
    s = solver_cls(wl, series_len=series_len or max(steps, 1), **kw)
    if init is not None:
        for c, a in init.items():
            s.set_field(c, a)
    s.step(steps)
    sim = oracle_from_workload(wl, initial=init, storage=storage)
    assert sim.dt == s.dt
    sim.run(steps)
    return s, sim


def _check_fields(s, sim, tol):
    for c in COMPS:
        ref = stored(sim, c)
        got = s.field(c)
        err = rel_l2(got, ref)
        assert err <= tol, (c, err)


def _check_probes(s, sim, tol, steps):
    if not sim.probes:
        return
    got = s.series(1, steps)
    ref = sim.series_array()
    for p in range(len(sim.probes)):
        err = rel_l2(got[:, p], ref[:, p])
        assert err <= tol, ("series", p, err)
    if len(s.wl.freqs):
        gd = s.dft()
        for p in range(len(sim.probes)):
            err = rel_l2(gd[p], sim.dft[p])
            assert err <= tol, ("dft", p, err)


def test_plain_pec_box_fp64_full():
    """The 32^3 FP64 PEC box, full size and step count."""
    import torch  # noqa
    from paper_2305_14176_amd.solver import YeeSolver
    wl = W.plain_pec_box()
    s, sim = _run_both(YeeSolver, wl, wl.steps)
    _check_probes(s, sim, TOL["f64"], wl.steps)
    _check_fields(s, sim, TOL["f64"])
    assert np.abs(s.series()).max() > 1e-3


@pytest.mark.parametrize("shape,cpml,v", [
    ((37, 29, 23), (4, 3, 5), "ragged rows"),
    ((100, 21, 18), (6, 2, 0), "no z layer"),
    ((200, 12, 30), (10, 5, 7), "four waves per row"),
    ((300, 9, 11), (6, 2, 3), "rows past 256: one sample per lane, five waves per row"),
    ((512, 6, 9), (6, 2, 3), "widest rows: eight waves per row, 16-wave workgroups"),
    ((2, 2, 2), (0, 0, 0), "smallest grid"),
])
def test_random_init_fp64_cpml(solver_cls, shape, cpml, v):
    nx, ny, nz = shape
    wl = W.cpml_block_lattice(n=nx, ny=ny, nz=nz, steps=12, precision="f64", cpml=0, nprobes=0, nfreq=0,
                              block=4)
    wl.cpml_cells = cpml
    wl.cpml_kappa_max = 2.0
    wl.cpml_alpha_max = 0.05
    wl.sources = [] if min(shape) < 4 else wl.sources
    s, sim = _run_both(solver_cls, wl, 12, init_seed=11)
    _check_fields(s, sim, TOL["f64"])


def test_fp64_two_samples_per_lane(solver_cls):
    """FP64 with two samples per lane (not the automatic choice: chosen
    explicitly), rows of 300 samples."""
    wl = W.cpml_block_lattice(n=300, ny=9, nz=11, steps=8, precision="f64", cpml=0, nprobes=0, nfreq=0, block=4)
    wl.cpml_cells = (6, 2, 3)
    wl.cpml_kappa_max = 2.0
    wl.cpml_alpha_max = 0.05
    s, sim = _run_both(solver_cls, wl, 8, init_seed=13, samples_per_lane=2)
    _check_fields(s, sim, TOL["f64"])


@pytest.mark.parametrize("shape,ty,kz,vpl", [
    ((256, 40, 33), 0, 0, 0),
    ((256, 40, 33), 3, 5, 0),
    ((256, 21, 19), 7, 3, 4),   # four samples per lane, one wave per row
    ((300, 17, 26), 3, 4, 2),   # two samples per lane, ragged row (12 waves, the two-sample limit)
    ((300, 17, 26), 0, 0, 0),   # automatic: two samples per lane, three waves per row
    ((160, 48, 48), 4, 16, 0),
    ((512, 9, 12), 1, 1, 0),    # widest rows (automatic: two samples per lane), one plane per chunk
    ((512, 9, 12), 0, 0, 1),    # widest rows, one sample per lane: eight waves, 16-wave workgroups
    ((512, 9, 12), 1, 2, 2),    # widest rows, two samples per lane
    ((512, 9, 12), 0, 0, 4),    # four samples per lane: automatic rows within its 8-wave limit
])
def test_random_init_fp32_launch_shapes(solver_cls, shape, ty, kz, vpl):
    nx, ny, nz = shape
    wl = W.cpml_block_lattice(n=nx, ny=ny, nz=nz, steps=10, precision="f32", cpml=1, nprobes=6, nfreq=8)
    wl.cpml_cells = (min(6, nx // 2), min(4, ny // 2), min(5, nz // 2))
    s, sim = _run_both(solver_cls, wl, 10, init_seed=12, tile_rows=ty, chunk_planes=kz, samples_per_lane=vpl)
    _check_fields(s, sim, TOL["f32"])


def test_cpml_lattice_fp32_probes_and_dft(solver_cls):
    """The CPML block-lattice workload at 64^3 (probes + DFT).

    At 200 steps (the pulse inside the grid) every output is gated at 1e-5
    against the FP64 oracle.  By 400 steps most of the pulse has left through
    the CPML and the fields compared are a decaying remainder; FP32 storage
    alone then moves the oracle itself by ~1e-5 from its FP64 run (storage
    rounded to FP32 each step, arithmetic FP64).  The 400-step outputs are
    gated at three times that drift, computed here, and all errors printed."""
    wl = W.cpml_block_lattice(n=64, steps=400)
    s, sim = _run_both(solver_cls, wl, 200, series_len=400)
    _check_probes(s, sim, TOL["f32"], 200)
    _check_fields(s, sim, TOL["f32"])
    s.step(200)
    sim.run(200)
    sim32 = oracle_from_workload(wl, storage="f32")
    sim32.run(400)
    ref = sim.series_array()
    drift = max([rel_l2(sim32.series_array()[:, p], ref[:, p]) for p in range(len(wl.probes))]
                + [rel_l2(stored(sim32, c), stored(sim, c)) for c in COMPS])
    got = s.series()
    es = max(rel_l2(got[:, p], ref[:, p]) for p in range(len(wl.probes)))
    ed = max(rel_l2(s.dft()[p], sim.dft[p]) for p in range(len(wl.probes)))
    ef = max(rel_l2(s.field(c), stored(sim, c)) for c in COMPS)
    _say(f"[gpu] fp32 64^3, 400 steps vs FP64 oracle: series {es:.2e} dft {ed:.2e} fields {ef:.2e}; "
         f"FP32-storage drift of the oracle itself {drift:.2e}")
    assert max(es, ed, ef) <= 3.0 * drift + 1e-6


def test_cpml_lattice_full_size_fp32_few_steps(solver_cls):
    """256^3 in the benchmark's launch shape, 3 steps from a random state."""
    wl = W.cpml_block_lattice(n=256, steps=3, nprobes=16)
    s, sim = _run_both(solver_cls, wl, 3, init_seed=21)
    _check_fields(s, sim, TOL["f32"])
    _check_probes(s, sim, TOL["f32"], 3)


def test_fp64_streamed_stores_few_steps(solver_cls):
    """160^3 in FP64: the twelve component arrays a step reads and writes
    (33 MB each) exceed the 256 MB last-level cache, so the step runs with its
    stores streamed past it; 3 steps from a random state with CPML, probes and
    the DFT, against the FP64 oracle."""
    wl = W.cpml_block_lattice(n=160, steps=3, precision="f64", nprobes=4, nfreq=8)
    s, sim = _run_both(solver_cls, wl, 3, init_seed=23)
    _check_fields(s, sim, TOL["f64"])
    _check_probes(s, sim, TOL["f64"], 3)


@pytest.mark.parametrize("steps", [1, 10])
def test_fp16_storage_few_steps(solver_cls, steps):
    """FP16 storage, few steps from a common random state: the GPU and the
    oracle emulating FP16 storage take the same rounding decisions except where
    FP32 and FP64 arithmetic straddle an fp16 rounding boundary."""
    wl = W.fp16_substrate(64, 64, 40, steps=steps, cpml=6)
    s, sim = _run_both(solver_cls, wl, steps, init_seed=31)
    _check_fields(s, sim, TOL["f16"])


def test_series_ring_and_dft_chunking(solver_cls):
    """A ring shorter than the run: the DFT is folded chunk by chunk."""
    wl = W.cpml_block_lattice(n=48, steps=150, nprobes=5, nfreq=16)
    s = solver_cls(wl, series_len=32)
    s.step(100)
    s.step(50)
    sim = oracle_from_workload(wl)
    sim.run(150)
    got = s.series(150 - 31, 32)
    ref = sim.series_array()[150 - 32:]
    for p in range(5):
        assert rel_l2(got[:, p], ref[:, p]) <= TOL["f32"]
    gd = s.dft()
    for p in range(5):
        assert rel_l2(gd[p], sim.dft[p]) <= TOL["f32"]
    with pytest.raises(Exception):
        s.series(1, 10)   # no longer in the ring


@pytest.mark.timeout(600)
def test_fp16_substrate_full_size_one_step(solver_cls):
    """512 x 512 x 256 with FP16 storage (the layered substrate with its PEC
    strip mask) in the benchmark's launch shape: one step from a random state
    (every update term, layer and mask is active) against the oracle emulating
    FP16 storage.  The oracle needs about a minute and 30 GB of host memory."""
    wl = W.fp16_substrate(steps=1)
    s, sim = _run_both(solver_cls, wl, 1, init_seed=41)
    _check_fields(s, sim, TOL["f16"])


@pytest.mark.parametrize("vpl", [0, 1])
def test_fp16_storage_wide_rows(solver_cls, vpl):
    """FP16 storage on rows of 300 samples: the automatic two samples per lane
    (three waves per row) and one sample per lane (five waves, 2-byte loads)."""
    wl = W.fp16_substrate(300, 40, 40, steps=4, cpml=4)
    s, sim = _run_both(solver_cls, wl, 4, init_seed=51, samples_per_lane=vpl)
    _check_fields(s, sim, TOL["f16"])


def test_fp32_fewer_planes_than_a_chunk(solver_cls):
    """nz below the smallest automatic chunk (one chunk, one warm-up-free march)."""
    wl = W.cpml_block_lattice(n=96, ny=50, nz=5, steps=6, precision="f32", cpml=1, nprobes=2, nfreq=4)
    wl.cpml_cells = (5, 4, 1)
    s, sim = _run_both(solver_cls, wl, 6, init_seed=52)
    _check_fields(s, sim, TOL["f32"])
    _check_probes(s, sim, TOL["f32"], 6)
