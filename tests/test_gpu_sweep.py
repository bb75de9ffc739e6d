"""GPU tests of the two-step sweep (two leapfrog steps per pass over the grid).

Every sample of a two-step sweep is computed with the same instruction
sequence as in a single step, so the sweep is compared with single steps
bitwise (fields, probe series) on the same context configuration, and with the
FP64 oracle at the usual tolerance.  The cases cover ragged rows, one, two and
four samples per lane, CPML on every axis with graded kappa and alpha, a PEC
plane mask, several sources (one inside a tile's halo), E and H probes, odd
step counts (a single step finishes the run), chunks shorter and longer than
the grid and FP16 storage.
"""
import sys

import numpy as np
import pytest

from paper_2305_14176_amd import workloads as W
from _helpers import oracle_from_workload, rel_l2, stored

pytestmark = pytest.mark.gpu

COMPS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def solver_cls():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_14176_amd.solver import YeeSolver
    return YeeSolver


def _case(nx, ny, nz, cpml, precision="f32", steps=9, nprobes=6, nfreq=8, pec=False, hprobe=True):
    wl = W.cpml_block_lattice(n=nx, ny=ny, nz=nz, steps=steps, precision=precision, cpml=0, nprobes=nprobes,
                              nfreq=nfreq, block=4)
    wl.cpml_cells = cpml
    wl.cpml_kappa_max = 1.7
    wl.cpml_alpha_max = 0.04
    if pec:
        mask = np.zeros((ny, nx), np.uint8)
        mask[ny // 4: ny // 2, nx // 5: nx // 2] = 3
        mask[ny // 2: ny // 2 + 2, :] |= 4
        wl.pec_planes = [(nz // 2, mask)]
    # a second source near a y-tile edge and an H probe
    src = wl.sources[0]
    wl.sources = [src, W.SourceSpec(1, nx // 3, min(ny - 2, 9), max(1, nz // 3), "gauss_deriv", 0.7,
                                    30.0, 9.0, 0.0, unit="dt")]
    if hprobe and len(wl.probes) >= 2:
        c, i, j, k = wl.probes[1]
        wl.probes[1] = (4, i, j, k)
    return wl


def _pair(solver_cls, wl, steps, init_seed, sweep_kw=None):
    init = W.random_initial_fields(wl, init_seed) if init_seed is not None else None
    out = []
    for mode in (1, 2):
        kw = dict(steps_per_sweep=mode)
        if mode == 2 and sweep_kw:
            kw.update(sweep_kw)
        s = solver_cls(wl, series_len=max(steps, 2), **kw)
        info = s.launch_info()
        assert info["steps_per_sweep"] == mode, info
        if init is not None:
            for c, a in init.items():
                s.set_field(c, a)
        _say(f"[gpu] sweep {wl.name} prec={wl.precision} steps={steps} mode={mode} launch={info}")
        s.step(steps)
        out.append(s)
    return out, init


def _check_bitwise(one, two, steps):
    for c in COMPS:
        np.testing.assert_array_equal(two.field(c), one.field(c), err_msg=c)
    if len(one.wl.probes):
        np.testing.assert_array_equal(two.series(1, steps), one.series(1, steps))
        if len(one.wl.freqs):
            assert rel_l2(two.dft(), one.dft()) <= 1e-13


@pytest.mark.parametrize("shape,cpml,steps,kw", [
    ((37, 29, 23), (4, 3, 5), 9, None),          # ragged rows, one sample per lane
    ((100, 21, 18), (6, 2, 0), 8, None),         # two samples per lane, no z layer
    ((200, 30, 40), (10, 5, 7), 11, None),       # four samples per lane, several y-tiles and chunks
    ((256, 20, 33), (10, 10, 10), 6, {"sweep_rows": 3, "sweep_planes": 4}),
    ((256, 20, 33), (10, 10, 10), 6, {"sweep_rows": 4, "sweep_planes": 64}),   # one chunk taller than the grid
    ((64, 12, 9), (0, 0, 0), 7, {"sweep_rows": 1, "sweep_planes": 1}),          # PEC box, one-row tiles
    ((2, 2, 2), (0, 0, 0), 5, None),             # smallest grid
])
def test_two_step_sweep_bitwise_equals_single_steps(solver_cls, shape, cpml, steps, kw):
    wl = _case(*shape, cpml=cpml, steps=steps, pec=min(shape) >= 8, nprobes=6 if min(shape) >= 8 else 0,
               nfreq=8 if min(shape) >= 8 else 0)
    if min(shape) < 4:
        wl.sources = []
    (one, two), _ = _pair(solver_cls, wl, steps, init_seed=7, sweep_kw=kw)
    _check_bitwise(one, two, steps)


def test_two_step_sweep_fp16_storage_bitwise(solver_cls):
    wl = W.fp16_substrate(96, 40, 44, steps=10, cpml=6)
    (one, two), _ = _pair(solver_cls, wl, 10, init_seed=9)
    _check_bitwise(one, two, 10)


@pytest.mark.parametrize("precision", ["f32", "f16"])
def test_two_step_sweep_streamed_stores_bitwise(solver_cls, precision):
    """Grids whose fields exceed the 256 MB last-level cache (256^3 FP32;
    256 x 256 x 192 with FP16 storage): the single steps and the sweeps both
    stream their stores past it.  5 steps (two sweeps, then a single step) from
    a random state, bitwise."""
    if precision == "f32":
        wl = W.cpml_block_lattice(n=256, steps=5)
    else:
        wl = W.fp16_substrate(256, 256, 192, steps=5, cpml=8)
    (one, two), _ = _pair(solver_cls, wl, 5, init_seed=13)
    _check_bitwise(one, two, 5)


@pytest.mark.parametrize("shape,cpml", [((150, 26, 31), (8, 6, 5)), ((256, 18, 25), (10, 4, 6))])
def test_two_step_sweep_against_oracle(solver_cls, shape, cpml):
    steps = 14
    wl = _case(*shape, cpml=cpml, steps=steps, pec=True)
    init = W.random_initial_fields(wl, 5)
    s = solver_cls(wl, series_len=steps, steps_per_sweep=2)
    for c, a in init.items():
        s.set_field(c, a)
    _say(f"[gpu] sweep vs oracle {wl.name} launch={s.launch_info()}")
    s.step(steps)
    sim = oracle_from_workload(wl, initial=init)
    sim.run(steps)
    for c in COMPS:
        assert rel_l2(s.field(c), stored(sim, c)) <= 1e-5, c
    got, ref = s.series(1, steps), sim.series_array()
    for p in range(len(wl.probes)):
        assert rel_l2(got[:, p], ref[:, p]) <= 1e-5, p
        assert rel_l2(s.dft()[p], sim.dft[p]) <= 1e-5, p


def test_two_step_sweep_availability(solver_cls):
    from paper_2305_14176_amd import _lib
    wl = W.cpml_block_lattice(n=64, steps=4)
    assert solver_cls(wl, steps_per_sweep=2).launch_info()["steps_per_sweep"] == 2
    with pytest.raises(_lib.YeeError):
        solver_cls(W.plain_pec_box(), steps_per_sweep=2)      # FP64 takes single steps
    wide = W.cpml_block_lattice(n=300, ny=8, nz=8, steps=2, nprobes=0, nfreq=0, cpml=2)
    with pytest.raises(_lib.YeeError):
        solver_cls(wide, steps_per_sweep=2)                   # rows past 256 samples
    assert solver_cls(wide).launch_info()["steps_per_sweep"] == 1
