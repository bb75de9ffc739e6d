"""Write the stored expected values of the long GPU parity runs.

Calls only the FP64 oracle (``oracle/``) and the seeded input generators: no
value here comes from the HIP library.  Each file holds, for one workload, the
probe series, the probe DFTs and the values of every component at a seeded
sample of stored positions (plus the positions themselves) at a few steps.

    python tests/golden/make_golden.py cpml256     # 256^3 FP32 workload, 1000 steps, FP64 oracle
                                                   # (about 90 minutes on one core)
    python tests/golden/make_golden.py fp16sub     # 128 x 128 x 64 substrate, 2000 steps, oracle
                                                   # emulating FP16 storage and the plain FP64 oracle
    python tests/golden/make_golden.py fp16sub_f32 # the same substrate, FP16 storage with FP32
                                                   # arithmetic (about 6 minutes)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

from paper_2305_14176_amd import workloads as W  # noqa: E402  (input generators only)
from _helpers import oracle_from_workload, stored  # noqa: E402

COMPS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")


def sample_points(wl, count, seed):
    """Seeded stored positions (i, j, k) per component, the probes' cells included."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = np.stack([rng.integers(0, wl.nx, count), rng.integers(0, wl.ny, count), rng.integers(0, wl.nz, count)], 1)
    extra = np.array([[i, j, k] for (_, i, j, k) in wl.probes], dtype=np.int64).reshape(-1, 3)
    return np.concatenate([extra, pts]).astype(np.int32)


def run(wl, storage, steps, pts, marks=(), arith="f64"):
    sim = oracle_from_workload(wl, storage=storage, arith=arith)
    t0 = time.time()
    out = {}
    for n in range(1, steps + 1):
        sim.step()
        if n in marks or n == steps:
            out[n] = {c: stored(sim, c)[pts[:, 0], pts[:, 1], pts[:, 2]].copy() for c in COMPS}
            out[n]["_norm"] = {c: float(np.linalg.norm(stored(sim, c))) for c in COMPS}
            out[n]["_full"] = {c: stored(sim, c).copy() for c in COMPS} if n == steps else None
        if n % 100 == 0:
            print(f"  {wl.name} {storage}: step {n}/{steps}, {time.time() - t0:.0f} s", flush=True)
    return sim, out


def cpml256():
    # the full workload: the pulse peaks inside the grid around step 200 and
    # reaches every probe before step 1000; fields are kept at 300 and 1000
    steps = 1000
    wl = W.cpml_block_lattice(n=256, steps=steps)
    pts = sample_points(wl, 8192, seed=2002)
    sim, out = run(wl, "f64", steps, pts, marks=(300,))
    fields = {}
    for n in sorted(out):
        fields.update({f"field_{c}_{n}": out[n][c] for c in COMPS})
        fields.update({f"norm_{c}_{n}": out[n]["_norm"][c] for c in COMPS})
    np.savez_compressed(os.path.join(HERE, "cpml_block_lattice_256_1000steps.npz"),
                        steps=steps, marks=np.array(sorted(out)), points=pts, series=sim.series_array(),
                        dft=np.array(sim.dft), **fields)


def fp16sub():
    steps = 2000
    wl = W.fp16_substrate(128, 128, 64, steps=steps)
    pts = sample_points(wl, 4096, seed=3003)
    marks = (500, 1000, 1500)
    s16, o16 = run(wl, "f16", steps, pts, marks)
    s64, o64 = run(wl, "f64", steps, pts, marks)
    rec = {}
    # the error of FP16 storage itself: the oracle's FP16 emulation against FP64 (relative L2 over the
    # whole component at the marks, per probe series and DFT at the end)
    for n in sorted(o16):
        for c in COMPS:
            if o16[n]["_full"] is not None:
                d = np.linalg.norm(o16[n]["_full"][c] - o64[n]["_full"][c]) / np.linalg.norm(o64[n]["_full"][c])
                rec[f"emul_vs_f64_field_{c}_{n}"] = d
    a16, a64 = s16.series_array(), s64.series_array()
    rec["emul_vs_f64_series"] = np.array([np.linalg.norm(a16[:, p] - a64[:, p]) / np.linalg.norm(a64[:, p])
                                          for p in range(a64.shape[1])])
    rec["emul_vs_f64_dft"] = np.array([np.linalg.norm(s16.dft[p] - s64.dft[p]) / np.linalg.norm(s64.dft[p])
                                       for p in range(a64.shape[1])])
    # sampled fields in float32: the emulated values are fp16 numbers times a
    # power of two (exact in float32); the FP64 ones keep 2^-24 relative, far
    # below the errors compared against them
    fields = {}
    for n in sorted(o16):
        for c in COMPS:
            fields[f"f16_{c}_{n}"] = o16[n][c].astype(np.float32)
            fields[f"f64_{c}_{n}"] = o64[n][c].astype(np.float32)
    np.savez_compressed(os.path.join(HERE, "fp16_substrate_128x128x64_2000steps.npz"),
                        steps=steps, marks=np.array(sorted(o16)), points=pts,
                        series_f16=a16, series_f64=a64, dft_f16=np.array(s16.dft), dft_f64=np.array(s64.dft),
                        **fields, **rec)
    print({k: (float(np.max(v)) if np.ndim(v) else float(v)) for k, v in rec.items()})


def fp16sub_f32():
    # the substrate of fp16sub (same sample positions and marks), FP16 storage
    # rounding the results of FP32 arithmetic, as the device path computes
    steps = 2000
    wl = W.fp16_substrate(128, 128, 64, steps=steps)
    pts = sample_points(wl, 4096, seed=3003)
    marks = (500, 1000, 1500)
    sim, out = run(wl, "f16", steps, pts, marks, arith="f32")
    fields = {f"f16a32_{c}_{n}": out[n][c].astype(np.float32) for n in sorted(out) for c in COMPS}
    np.savez_compressed(os.path.join(HERE, "fp16_substrate_128x128x64_2000steps_f32arith.npz"),
                        steps=steps, marks=np.array(sorted(out)), points=pts, series=sim.series_array(),
                        dft=np.array(sim.dft), **fields)


if __name__ == "__main__":
    {"cpml256": cpml256, "fp16sub": fp16sub, "fp16sub_f32": fp16sub_f32}[sys.argv[1]]()
