"""GPU parity on the long and full-size runs, against stored oracle results.

The expected values under ``tests/golden/`` were written by
``tests/golden/make_golden.py``, which calls only the FP64 oracle and the
seeded input generators.

* 256^3 FP32, 10-cell CPML, 16 probes, 64 DFT frequencies, 1000 steps (the
  full-size FP32 workload), in single steps and in two-step sweeps: every
  probe series and every probe's DFT vector to 1e-5 relative L2 (measured
  2.5e-6 and 1.7e-6); every component at 8192 seeded positions plus the
  probe cells at step 300 (the pulse inside the grid) and at step 1000 (most
  of it gone through the CPML), to 1e-5 relative L2 over the sampled set
  (measured at most 6.2e-6 and 3.7e-6) and element by element to
  |got - ref| <= 4 n 2^-24 A, A the component's largest sampled value at
  step 300.  The element bound is the error model of an FP32 run: per step
  each value is stored once in FP32 and updated with FP32 coefficients (Ca,
  Cb, the inverse cell size), each at most 2^-24 relative from the oracle's
  FP64 values; in a stable scheme these errors add at most linearly over n
  steps.  Measured: 0.20 of the bound at step 300 (Ex, 1.45e-5 A), 0.02 at
  step 1000.  The errors are written as JSON to the run's output folder
  (golden256_errors_*.json).

* FP16 storage, layered substrate at 128 x 128 x 64, 2000 steps: the
  oracle's FP16 emulation (FP64 arithmetic, each stored value rounded to
  fp16 x 2^s) and the plain FP64 oracle are both stored.  Over a long run
  the fp16 rounding noise of two runs decorrelates once a single rounding
  decision differs, so no two FP16 runs agree to 1e-3 in the fields or the
  series; what is fixed is how large the storage error itself is.  Gates:
  - each component at each of four times (relative L2 over 4096 sampled
    positions, an average over many samples): the GPU's error against FP64
    within 1.5 times the emulation's own error against FP64 (measured
    0.88-1.25), and GPU and emulation within 2.5 times that error of each
    other (two independent noises of one size differ by about sqrt(2) times
    it; measured 1.28-1.78);
  - probe series and DFT vectors: each probe's error is one realisation of
    the rounding noise, and two realisations differ by up to 2x per probe
    (measured 0.78-1.96), so the 16 probes are gated together: the RMS over
    probes of the GPU's error within 1.5 times that of the emulation
    (measured 1.04 series, 1.19 DFT), the worst probe within 2 times the
    emulation's worst (1.02, 1.12), and the RMS of GPU against emulation
    within 2.5 times the emulation's RMS (1.44, 1.59).
  A second emulation computes in FP32 (the device's arithmetic) before each
  fp16 rounding (`..._f32arith.npz`, same points and marks).  It differs
  from the FP64-arithmetic emulation by 1.0-1.4e-2 at step 500 and 3-6.5e-2
  at step 2000, about sqrt(2) times either one's error against FP64: the
  rounding noise of two FP16 runs decorrelates whatever their arithmetic, so
  a 1e-3 match between two FP16 runs is out of reach over a long run.  The
  GPU is gated against it like against the other emulation (within 2.5
  times the storage error).
  The measured curve is written as JSON to the run's output folder
  (fp16_error_curve.json).
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_2305_14176_amd import workloads as W
from _helpers import rel_l2

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
ROOT = os.path.dirname(HERE)
COMPS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")
ELEMENT_UNITS = 4    # FP32 roundings per value and step in the element bound of the 256^3 run


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def solver_cls():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_14176_amd.solver import YeeSolver
    return YeeSolver


def _load(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{path} is missing: run python tests/golden/make_golden.py")
    return np.load(path, allow_pickle=False)


def _sample(s, pts):
    return {c: s.field(c)[pts[:, 0], pts[:, 1], pts[:, 2]] for c in COMPS}


@pytest.mark.parametrize("steps_per_sweep", [1, 2])
def test_cpml_lattice_256_fp32_full_run(solver_cls, steps_per_sweep):
    g = _load("cpml_block_lattice_256_1000steps.npz")
    steps = int(g["steps"])
    marks = [int(m) for m in g["marks"]]
    wl = W.cpml_block_lattice(n=256, steps=steps)
    s = solver_cls(wl, series_len=steps, steps_per_sweep=steps_per_sweep)
    _say(f"[gpu] golden 256^3 fp32 {steps} steps, fields at {marks}, launch={s.launch_info()}")
    pts = g["points"]
    ncell = wl.nx * wl.ny * wl.nz
    rms300 = {c: float(g[f"norm_{c}_300"]) / np.sqrt(ncell) for c in COMPS}
    amp300 = {c: float(np.abs(g[f"field_{c}_300"]).max()) for c in COMPS}
    rec = {"workload": "cpml_block_lattice 256^3 FP32, CPML 10, 1000 steps", "steps_per_sweep": steps_per_sweep,
           "fields": {}}
    failures = []
    done = 0
    for m in marks:
        s.step(m - done)
        done = m
        got = _sample(s, pts)
        row = {}
        for c in COMPS:
            ref = g[f"field_{c}_{m}"]
            d = np.abs(got[c] - ref)
            bound = ELEMENT_UNITS * m * 2.0 ** -24 * amp300[c]
            row[c] = {"max_err_over_bound": float(d.max() / bound),
                      "max_err_over_rms300": float(d.max() / rms300[c]),
                      "max_err_over_max_ref": float(d.max() / np.abs(ref).max()),
                      "rel_l2": float(rel_l2(got[c], ref))}
            if d.max() > bound:
                failures.append((m, c, "element", row[c]))
            if row[c]["rel_l2"] > 1e-5:
                failures.append((m, c, "rel_l2", row[c]))
        rec["fields"][m] = row
        _say(f"[gpu]   step {m}: worst element error / bound: "
             + " ".join(f"{c} {row[c]['max_err_over_bound']:.2f}" for c in COMPS)
             + "; relative L2: " + " ".join(f"{c} {row[c]['rel_l2']:.1e}" for c in COMPS))
    got_series, got_dft = s.series(1, steps), s.dft()
    es = [float(rel_l2(got_series[:, p], g["series"][:, p])) for p in range(len(wl.probes))]
    ed = [float(rel_l2(got_dft[p], g["dft"][p])) for p in range(len(wl.probes))]
    rec["series_rel_l2"], rec["dft_rel_l2"] = es, ed
    _say(f"[gpu]   worst probe series {max(es):.2e}, worst DFT {max(ed):.2e}")
    out = os.path.join(ROOT, "gpurun_out")
    os.makedirs(out, exist_ok=True)
    with open(os.path.join(out, f"golden256_errors_sweep{steps_per_sweep}.json"), "w") as f:
        json.dump(rec, f, indent=1)
    if max(es) > 1e-5 or max(ed) > 1e-5:
        failures.append(("series/dft", max(es), max(ed)))
    assert not failures, failures
    # the pulse reached every probe: in the oracle's run each probe peaks
    # between steps 636 and 972, at 3.7e-5 to 2.5e-4
    assert min(np.abs(g["series"]).max(axis=0)) > 1e-5


def test_fp16_substrate_2000_steps_error_curve(solver_cls):
    g = _load("fp16_substrate_128x128x64_2000steps.npz")
    g32 = _load("fp16_substrate_128x128x64_2000steps_f32arith.npz")    # same points and marks
    assert np.array_equal(g32["points"], g["points"])
    steps = int(g["steps"])
    marks = [int(m) for m in g["marks"]]
    wl = W.fp16_substrate(128, 128, 64, steps=steps)
    s = solver_cls(wl, series_len=steps)
    pts = g["points"]
    _say(f"[gpu] golden fp16 substrate 128x128x64 {steps} steps, marks {marks}")
    curve = {"workload": "fp16 substrate 128x128x64, 2000 steps", "fp16_exp": list(wl.fp16_exp), "marks": {}}
    failures = []
    done = 0
    for m in marks:
        s.step(m - done)
        done = m
        got = _sample(s, pts)
        row = {}
        for c in COMPS:
            f16, f64 = g[f"f16_{c}_{m}"], g[f"f64_{c}_{m}"]
            o = float(rel_l2(f16, f64))       # the storage error itself (oracle emulation vs FP64)
            e64 = float(rel_l2(got[c], f64))
            e16 = float(rel_l2(got[c], f16))
            row[c] = {"gpu_vs_f64": e64, "gpu_vs_emulation": e16, "emulation_vs_f64": o}
            if m in [int(v) for v in g32["marks"]]:
                a32 = g32[f"f16a32_{c}_{m}"]
                row[c]["gpu_vs_fp32_emulation"] = float(rel_l2(got[c], a32))
                row[c]["fp32_emulation_vs_emulation"] = float(rel_l2(a32, f16))
                if row[c]["gpu_vs_fp32_emulation"] > 2.5 * o:
                    failures.append((m, c, "fp32 emulation", row[c]))
            if e64 > 1.5 * o or e16 > 2.5 * o:
                failures.append((m, c, e64, e16, o))
        curve["marks"][m] = row
        _say(f"[gpu]   step {m}: " + " ".join(f"{c} {row[c]['gpu_vs_f64']:.2e}/{row[c]['emulation_vs_f64']:.2e}"
                                          for c in COMPS))
    got_series, got_dft = s.series(1, steps), s.dft()
    for name, got_all, a16, a64 in (("series", got_series.T, g["series_f16"].T, g["series_f64"].T),
                                    ("dft", got_dft, g["dft_f16"], g["dft_f64"])):
        rows = []
        for p in range(len(wl.probes)):
            o = float(rel_l2(a16[p], a64[p]))
            e64 = float(rel_l2(got_all[p], a64[p]))
            e16 = float(rel_l2(got_all[p], a16[p]))
            rows.append({"gpu_vs_f64": e64, "gpu_vs_emulation": e16, "emulation_vs_f64": o})
        curve[name] = rows
        rms = {k: float(np.sqrt(np.mean([r[k] ** 2 for r in rows]))) for k in rows[0]}
        worst = {k: max(r[k] for r in rows) for k in rows[0]}
        curve[name + "_rms_over_probes"] = rms
        if (rms["gpu_vs_f64"] > 1.5 * rms["emulation_vs_f64"] or worst["gpu_vs_f64"] > 2.0 * worst["emulation_vs_f64"]
                or rms["gpu_vs_emulation"] > 2.5 * rms["emulation_vs_f64"]):
            failures.append((name, rms, worst))
        _say(f"[gpu]   {name}: worst gpu vs f64 {max(r['gpu_vs_f64'] for r in rows):.2e}, worst emulation vs f64 "
             f"{max(r['emulation_vs_f64'] for r in rows):.2e}, worst gpu vs emulation "
             f"{max(r['gpu_vs_emulation'] for r in rows):.2e}")
    out = os.path.join(ROOT, "gpurun_out")
    os.makedirs(out, exist_ok=True)
    with open(os.path.join(out, "fp16_error_curve.json"), "w") as f:
        json.dump(curve, f, indent=1)
    assert not failures, failures
    assert min(np.abs(got_series[:, p]).max() for p in range(len(wl.probes))) > 1e-4   # the pulse arrived

