"""Benchmark of the Yee FDTD step on one MI355X.

Workload: the 256^3 FP32 grid with a 10-cell CPML on all faces, an 8^3-cell
block lattice (eps_r ~ U[1, 10), sigma ~ U[0, 0.1) S/m), a modulated-Gaussian
Ez source, 16 probes and a 64-frequency FP64 running DFT.  One "step" is one
full leapfrog step (H and E half-updates, CPML, source, probes; the DFT fold
runs on the same stream inside the timed region).

Prints one JSON line: Mcell-updates/s, the HBM roofline of the fused step
kernel (algorithmic bytes per launch over its measured duration), and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak (AMD public spec)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_cpml256_fp32_traffic.json")
COPY_MIB = 512                 # size of the calibration copy in --profile-run


def algorithmic_bytes_per_step(wl, elem_bytes=4, psi_bytes=4):
    """Bytes one step must move at minimum: every field component read and
    written once (12 component accesses per cell) plus every CPML auxiliary
    read and written once.  The material table (32^3 blocks) stays in cache."""
    nx, ny, nz = wl.nx, wl.ny, wl.nz
    fields = 12 * elem_bytes * nx * ny * nz
    lx, ly, lz = wl.cpml_cells
    psi_elems = 2 * (nz * ny * 2 * lx) + 2 * (nz * 2 * ly * nx) + 2 * (2 * lz * ny * nx)  # per side
    psi = 2 * 2 * psi_bytes * psi_elems     # E side + H side, read + write
    return fields + psi, fields, psi


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("yee_kernels.hpp", "yee_runtime.hip"):
        with open(os.path.join(ROOT, "paper_2305_14176_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic():
    """Counter-measured HBM bytes per launch, if taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(wl, budget_s=15.0, max_steps=5):
    """The FP64 oracle (numpy, single thread) on the same 256^3 workload, a few steps."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _helpers import oracle_from_workload
    sim = oracle_from_workload(wl)
    sim.step()  # first step pays page faults of the large arrays
    t0 = time.perf_counter()
    n = 0
    while n < max_steps:
        sim.step()
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": wl.cells * n / dt / 1e6, "unit": "Mcell-updates/s", "cores": 1, "host_cores": os.cpu_count(),
            "kind": "oracle",
            "sample": f"{n} steps of the same {wl.nx}x{wl.ny}x{wl.nz} workload after 1 untimed step "
                      f"(numpy FP64, single-threaded elementwise: 1 of {os.cpu_count()} host cores), {dt:.1f} s"}


def serving_benchmark(n_requests=64, loads=(0.8, 1.2), seed=4, steps_per_replay=32, max_slots=32,
                      hbm_budget=4 << 30, sample=16, max_active_cells="default"):
    """Serving sweep: Poisson arrivals at `load` x the plain one-at-a-time capacity.

    Requests follow the serving workload (cubic sides from {32, 48, 64, 96, 128,
    160}, 500-3000 steps, CPML 8, FP32, seeded).  The plain capacity C (requests/s)
    is measured on the first `sample` requests served back to back; arrivals then
    come at rate load * C.  Both the plain first-come-first-served loop and the
    batched server see the same arrival times.
    """
    import numpy as np
    from paper_2305_14176_amd import workloads as W
    from paper_2305_14176_amd.serving import BatchServer, Request, serve_one_at_a_time

    if max_active_cells == "default":
        from paper_2305_14176_amd.serving import DEFAULT_ACTIVE_CELLS
        max_active_cells = DEFAULT_ACTIVE_CELLS
    gaps, wls = W.serving_sweep(n_requests, seed=seed)
    cells = [w.cells * w.steps for w in wls]

    def make(arrivals):
        return [Request(w, arrival=float(t), rid=i) for i, (w, t) in enumerate(zip(wls, arrivals))]

    # warm-up: two requests through each path, untimed (first launches, memory
    # pools and the batch's graph capture would otherwise count against the
    # capacity that sets the arrival rates)
    serve_one_at_a_time(make(np.zeros(n_requests))[:2])
    srv = BatchServer(max_slots=max_slots, hbm_budget=hbm_budget, steps_per_replay=steps_per_replay,
                      max_active_cells=max_active_cells)
    srv.serve(make(np.zeros(n_requests))[:2])
    srv.close()
    # closed-loop capacities on the first `sample` requests (all present at t = 0)
    t0 = time.perf_counter()
    serve_one_at_a_time(make(np.zeros(n_requests))[:sample])
    cap = sample / (time.perf_counter() - t0)
    srv = BatchServer(max_slots=max_slots, hbm_budget=hbm_budget, steps_per_replay=steps_per_replay,
                      max_active_cells=max_active_cells)
    t0 = time.perf_counter()
    srv.serve(make(np.zeros(n_requests))[:sample])
    cap_b = sample / (time.perf_counter() - t0)
    srv.close()
    # open loop: the same Poisson arrivals for both, at each load
    runs = {}
    for load in loads:
        arrivals = np.asarray(gaps) / (load * cap)
        plain = serve_one_at_a_time(make(arrivals))
        srv = BatchServer(max_slots=max_slots, hbm_budget=hbm_budget, steps_per_replay=steps_per_replay,
                          max_active_cells=max_active_cells)
        batched = srv.serve(make(arrivals))
        srv.close()
        runs[load] = (plain, batched, srv.replays)

    def stats(done):
        lat = np.array([r.latency for r in done])
        makespan = max(r.finished for r in done)
        return {"p50_latency_s": round(float(np.percentile(lat, 50)), 4),
                "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
                "mean_latency_s": round(float(lat.mean()), 4),
                "makespan_s": round(float(makespan), 3),
                "mcell_updates_per_s": round(sum(cells) / makespan / 1e6, 1)}

    out = {"requests": n_requests, "plain_capacity_req_per_s": round(cap, 3),
           "batched_capacity_req_per_s": round(cap_b, 3),
           "steps_per_replay": steps_per_replay, "max_slots": max_slots, "hbm_budget_bytes": hbm_budget,
           "max_active_cells": max_active_cells,
           "workload": "serving_request: side in {32,48,64,96,128,160}, 500-3000 steps, CPML 8, FP32"}
    for load, (plain, batched, replays) in runs.items():
        out[f"load_{load}"] = {"arrival_rate_req_per_s": round(load * cap, 3), "batched": stats(batched),
                               "plain_fifo": stats(plain), "replays": replays}
    return out


def copy_bandwidth(mib=1024, reps=20):
    """A practical HBM ceiling on this device: a plain device-to-device copy of
    `mib` MiB (read + write bytes per second, best of `reps`)."""
    import torch
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    nbytes = 2 * src.numel() * 4
    del src, dst
    torch.cuda.empty_cache()
    return nbytes / (best / 1e3) / 1e9


def precision_benchmark(steps=100, warmup=10):
    """The other precision modes at their configurations: FP16 storage
    (FP32 arithmetic, FP64 DFT) on the 512 x 512 x 256 layered substrate with a
    PEC strip mask, and FP64 on the 32^3 PEC box."""
    import torch
    from paper_2305_14176_amd import workloads as W
    from paper_2305_14176_amd.solver import YeeSolver
    out = {}
    for wl, eb, n in ((W.fp16_substrate(), 2, steps), (W.plain_pec_box(seed=1), 8, 200)):
        solver = YeeSolver(wl, device="cuda:0", series_len=max(1000, n))
        stream = torch.cuda.current_stream()
        solver.step(warmup)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        solver.step(n)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / n
        alg, fields_b, psi_b = algorithmic_bytes_per_step(wl, elem_bytes=eb, psi_bytes=8 if eb == 8 else 4)
        gbs = alg / (ms / 1e3) / 1e9
        out[wl.name] = {"dtype": {2: "f16 storage, f32 math, f64 dft", 8: "f64"}[eb], "steps": n,
                        "ms_per_step": round(ms, 5), "mcell_updates_per_s": round(wl.cells / (ms / 1e3) / 1e6, 1),
                        "algorithmic_bytes_per_step": alg, "hbm_gbs_algorithmic": round(gbs, 1),
                        "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
        solver.close()
        del solver
        torch.cuda.empty_cache()
    return out


def precision_errors():
    """Error of each output against the FP64 oracle, from the oracle results
    stored under tests/golden/ (written by tests/golden/make_golden.py):
    FP32 on the 256^3 CPML workload over its 1000 steps, and FP16 storage on the
    128 x 128 x 64 layered substrate over 2000 steps (with the error of the
    oracle's own FP16-storage emulation beside it)."""
    import numpy as np
    from paper_2305_14176_amd import workloads as W
    from paper_2305_14176_amd.solver import YeeSolver
    comps = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")

    def rel(x, r):
        x, r = np.asarray(x), np.asarray(r)
        return float(np.linalg.norm((x - r).ravel()) / np.linalg.norm(r.ravel()))

    def sample(s, pts):
        return {c: s.field(c)[pts[:, 0], pts[:, 1], pts[:, 2]] for c in comps}

    out = {}
    g = np.load(os.path.join(ROOT, "tests", "golden", "cpml_block_lattice_256_1000steps.npz"))
    steps = int(g["steps"])
    wl = W.cpml_block_lattice(n=256, steps=steps)
    s = YeeSolver(wl, device="cuda:0", series_len=steps)
    fields, done = {}, 0
    for m in [int(v) for v in g["marks"]]:
        s.step(m - done)
        done = m
        got = sample(s, g["points"])
        # element bound of an FP32 run: 4 n 2^-24 times the component's
        # largest sampled value at step 300 (the pulse inside the grid)
        bound = {c: 4 * m * 2.0 ** -24 * float(np.abs(g[f"field_{c}_300"]).max()) for c in comps}
        fields[m] = {c: {"sampled_rel_l2": round(rel(got[c], g[f"field_{c}_{m}"]), 9),
                         "worst_element_over_fp32_bound":
                             round(float(np.abs(got[c] - g[f"field_{c}_{m}"]).max() / bound[c]), 4)}
                     for c in comps}
    ser, dft = s.series(1, steps), s.dft()
    out[f"{wl.name}_fp32_{steps}_steps"] = {
        "series_rel_l2_max": max(rel(ser[:, p], g["series"][:, p]) for p in range(len(wl.probes))),
        "dft_rel_l2_max": max(rel(dft[p], g["dft"][p]) for p in range(len(wl.probes))),
        "fields_by_step": fields, "points": int(len(g["points"])), "reference": "FP64 oracle"}
    s.close()
    g = np.load(os.path.join(ROOT, "tests", "golden", "fp16_substrate_128x128x64_2000steps.npz"))
    steps = int(g["steps"])
    wl = W.fp16_substrate(128, 128, 64, steps=steps)
    s = YeeSolver(wl, device="cuda:0", series_len=steps)
    curve, done = {}, 0
    for m in [int(v) for v in g["marks"]]:
        s.step(m - done)
        done = m
        got = sample(s, g["points"])
        curve[m] = {c: {"gpu": round(rel(got[c], g[f"f64_{c}_{m}"]), 6),
                        "oracle_fp16_emulation": round(rel(g[f"f16_{c}_{m}"], g[f"f64_{c}_{m}"]), 6)}
                    for c in comps}
    ser, dft = s.series(1, steps), s.dft()
    npr = len(wl.probes)
    out[f"fp16_substrate_128x128x64_{steps}_steps"] = {
        "series_rel_l2_max": {"gpu": max(rel(ser[:, p], g["series_f64"][:, p]) for p in range(npr)),
                              "oracle_fp16_emulation": max(rel(g["series_f16"][:, p], g["series_f64"][:, p])
                                                           for p in range(npr))},
        "dft_rel_l2_max": {"gpu": max(rel(dft[p], g["dft_f64"][p]) for p in range(npr)),
                           "oracle_fp16_emulation": max(rel(g["dft_f16"][p], g["dft_f64"][p]) for p in range(npr))},
        "fields_sampled_rel_l2_by_step": curve, "points": int(len(g["points"])),
        "reference": "FP64 oracle"}
    s.close()
    return out


def adjoint_benchmark(checkpoint_every=64):
    """Gradient of the 128^3 design workload (FP32 fields, FP64 gradient):
    forward run with checkpoints, backward run (recompute + reverse steps),
    against the same N plain steps, with the default history budget; then
    the same gradient keeping the E history of only the newest segment, and
    of the newest half of the segments (the rest recomputed)."""
    import torch
    from paper_2305_14176_amd import workloads as W
    from paper_2305_14176_amd.adjoint import DesignProblem
    wl = W.adjoint_design()
    d0, d1 = wl.design
    box = (d0, d1, d0, d1, d0, d1)

    def timed(history_segments):
        prob = DesignProblem(wl, box, checkpoint_every=checkpoint_every, history_segments=history_segments)
        eps0 = prob.initial_design
        prob.forward(eps0)
        prob.gradient()              # warm-up of both passes
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob.forward(eps0)           # synchronizes (returns J to the host)
        t1 = time.perf_counter()
        g = prob.gradient()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        prob.solver.reset()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        prob.solver.step(prob.n_steps)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        res = (t1 - t0, t2 - t1, t4 - t3, g.numel(), prob.run.footprint, prob.n_steps, prob.run.history_segments)
        prob.close()
        return res

    # the default schedule: checkpoints every K steps, the newest segments'
    # E histories kept within the default history budget, the older
    # segments recomputed from their checkpoints
    fwd, bwd, plain, nbox, ws, n_steps, kept = timed(None)
    segments = -(-n_steps // checkpoint_every)
    out = {"workload": f"{wl.name}: design [{d0},{d1})^3, {n_steps} steps, {len(wl.probes)} Ez probes, "
                       f"checkpoint every {checkpoint_every}",
           "dtype": "f32 fields, f64 gradient",
           "schedule": f"{segments} segments: E history kept from the forward run for the newest {kept}, "
                       f"{segments - kept} recomputed from their checkpoints",
           "forward_ms": round(fwd * 1e3, 2), "backward_ms": round(bwd * 1e3, 2),
           "gradient_ms": round((fwd + bwd) * 1e3, 2), "plain_forward_ms": round(plain * 1e3, 2),
           "gradient_over_plain": round((fwd + bwd) / plain, 3),
           "design_cells": nbox, "workspace_bytes": ws}
    for name, h in (("one_history_kept", 1), ("half_history_kept", max(1, segments // 2))):
        fwd, bwd, plain, _, ws, _, _ = timed(h)
        out[name] = {"forward_ms": round(fwd * 1e3, 2), "backward_ms": round(bwd * 1e3, 2),
                     "gradient_ms": round((fwd + bwd) * 1e3, 2),
                     "gradient_over_plain": round((fwd + bwd) / plain, 3), "workspace_bytes": ws}
    return out


FP32_MFMA_PEAK_TFLOPS = 157.3     # published MI355X dense FP32 matrix peak
FP16_MFMA_PEAK_TFLOPS = 2500.0    # published MI355X dense fp16 matrix peak
FLOPS_PER_TERM = 8                # per (ray, sample): a complex multiply-add, four real multiply-adds
FP32_VECTOR_PEAK_TFLOPS = 157.3   # published MI355X FP32 vector peak
SPREAD_FLOPS_PER_RAY_BLOCK = 2 * 36 + 16 + 16   # per (ray, pair, chirp): 36 FMAs (8 taps), 16 mul, 16 grid adds
SPREAD_ATOMICS_PER_RAY_BLOCK = 16   # 64-bit LDS integer atomics per (ray, pair, chirp): 8 taps x (re, im)
# LDS: 128 bytes per clock per CU, 256 CUs at 2.4 GHz; one 64-bit atomic moves 8 bytes
LDS_ATOMIC64_PEAK_PER_S = 256 * 2.4e9 * 128 / 8


def sparams_benchmark():
    """Two-run S-parameters on the PEC-waveguide workloads (12 x 12 x 140
    cells, 6000 FP32 steps each): the GPU time of every run (HIP events on the
    launch stream), the host time of the extraction from the probe DFTs
    (yee_sparams), and the physical checks: the PEC short reflects fully
    (|S11| = 1) and the lossless slab conserves power (|S11|^2 + |S21|^2 = 1),
    over 44-66 GHz."""
    import numpy as np
    import torch
    from paper_2305_14176_amd import sparams as L
    from paper_2305_14176_amd import workloads as W
    from paper_2305_14176_amd.solver import YeeSolver
    ports = [([0], [1.0]), ([1], [1.0])]
    dft, run_ms = {}, {}
    for kind in ("ref", "short", "slab"):
        wl = W.waveguide_ports(kind, precision="f32")
        s = YeeSolver(wl, device="cuda:0")
        stream = torch.cuda.current_stream()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        s.step(wl.steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        run_ms[kind] = round(ev0.elapsed_time(ev1), 3)
        dft[kind] = s.dft()
        s.close()
    t0 = time.perf_counter()
    _, _, s_short = L.sparams(dft["ref"], dft["short"], ports)
    _, _, s_slab = L.sparams(dft["ref"], dft["slab"], ports)
    host_us = (time.perf_counter() - t0) / 2 * 1e6
    wl = W.waveguide_ports("ref")
    return {
        "workload": f"{wl.name}: PEC waveguide, CPML on the z faces, {wl.steps} FP32 steps, "
                    f"{len(wl.freqs)} frequencies 44-66 GHz, ports = Ez probes at k = 60 and 110",
        "run_ms": run_ms,
        "steps_per_s": round(wl.steps / (run_ms["ref"] / 1e3), 1),
        "extraction_us_host": round(host_us, 1),
        "short_max_abs_s11_minus_1": round(float(np.abs(np.abs(s_short[0]) - 1).max()), 5),
        "slab_max_power_error": round(float(np.abs(np.abs(s_slab[0]) ** 2 + np.abs(s_slab[1]) ** 2 - 1).max()), 5),
    }


def _time_cube(syn, ds, reps):
    """Average milliseconds of one whole IF cube (all chirp batches) over
    `reps` back-to-back calls on the current stream, after one untimed call."""
    import torch
    stream = torch.cuda.current_stream()
    syn.run(0, ds.amp)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        syn.run(0, ds.amp)
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


def if_synthesis_benchmark(reps=5, cpu=True, cpu_rays=1 << 15):
    """IF cube from ray meta data (Eqs. 1-7) on the full pedestrian scene:
    2^20 rays, 8 meshes x 4096 triangles, 12 antenna pairs, 128 chirps x 512
    samples, with the spreading method (rmd_if_cube) and the direct method
    (rmd_if_cube_direct); then the range-Doppler map of the cube (Eq. 4)."""
    import torch
    from paper_2305_14176_amd import raymeta as RM
    from paper_2305_14176_amd import rayscene as RS
    sc = RS.pedestrian_scene()
    ds = RM.DeviceScene(sc, device="cuda:0")
    r = sc.radar
    terms = sc.n_rays * sc.n_pairs * r.n_chirps * r.n_samples
    ray_blocks = sc.n_rays * sc.n_pairs * r.n_chirps
    syn = RM.Synthesizer(ds, method="spread")
    ms = _time_cube(syn, ds, reps)
    spec = torch.empty_like(syn.out)
    stream = torch.cuda.current_stream()
    RM.range_doppler(syn.out, out=spec)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(20):
        RM.range_doppler(syn.out, out=spec)
    ev1.record(stream)
    torch.cuda.synchronize()
    rd_ms = ev0.elapsed_time(ev1) / 20
    syn_d = RM.Synthesizer(ds, method="direct")
    ms_d = _time_cube(syn_d, ds, reps)
    spread_tflops = ray_blocks * SPREAD_FLOPS_PER_RAY_BLOCK / (ms / 1e3) / 1e12
    tflops_d = terms * FLOPS_PER_TERM / (ms_d / 1e3) / 1e12
    out = {
        "workload": f"{sc.name}: {sc.n_hits} hits, {sc.n_pairs} antenna pairs (3 TX x 4 RX), "
                    f"{r.n_chirps} chirps x {r.n_samples} samples, 77 GHz, B = 1 GHz, T_c = 51.2 us, f_s = 10 MHz",
        "method": "spread: type-1 non-uniform FFT (8-cell exponential-of-semicircle kernel on a 1024-cell grid, "
                  "64-bit fixed-point spreading with integer LDS atomics, FP64 partition sums, inverse DFT and "
                  "deconvolution)",
        "dtype": "f64 geometry and phases, f32 phasors and kernel values, i64 grid sums, f64 transform",
        "metric": "IF terms/s (ray x antenna pair x chirp x sample)",
        "value": round(terms / (ms / 1e3), 1),
        "unit": "terms/s",
        "ms_per_cube": round(ms, 3),
        "cubes_per_s": round(1e3 / ms, 3),
        "reps": reps,
        "range_doppler_ms": round(rd_ms, 4),
        "roofline": {"bound": "alu", "achieved": round(spread_tflops, 2), "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(spread_tflops / FP32_VECTOR_PEAK_TFLOPS, 4),
                     "peak_basis": "published FP32 vector peak (packed FMA); built without packed FP32, the issue "
                                   "limit is half of it",
                     "traffic": None, "algorithmic_flops_per_launch": ray_blocks * SPREAD_FLOPS_PER_RAY_BLOCK,
                     "flops_counted": "per ray, pair and chirp: 8 kernel values (36 FMAs), 16 multiplies, 16 grid "
                                      "additions; the FP64 antenna legs, conversions and atomics are not counted",
                     "lds_atomic_bound": {
                         "achieved_per_s": round(ray_blocks * SPREAD_ATOMICS_PER_RAY_BLOCK / (ms / 1e3), 1),
                         "peak_per_s": LDS_ATOMIC64_PEAK_PER_S,
                         "frac": round(ray_blocks * SPREAD_ATOMICS_PER_RAY_BLOCK / (ms / 1e3)
                                       / LDS_ATOMIC64_PEAK_PER_S, 4),
                         "basis": "16 64-bit integer LDS atomics per ray, pair and chirp against 128 B per clock "
                                  "per CU of LDS bandwidth (8 B per atomic, no bank conflicts)"},
                     "kernel": "rmd::spread_kernel (timed with rmd::geometry_kernel and rmd::finish_kernel: "
                               "one IF cube)",
                     "kernel_ms_avg": round(ms, 3)},
        "direct": {
            "method": "direct: fp16 hi/lo split MFMA products (rmd_if_cube_direct)",
            "value": round(terms / (ms_d / 1e3), 1), "unit": "terms/s", "ms_per_cube": round(ms_d, 3),
            "roofline": {"bound": "mfma", "achieved": round(3 * tflops_d, 2), "peak": FP16_MFMA_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(3 * tflops_d / FP16_MFMA_PEAK_TFLOPS, 4),
                         "peak_basis": "dense fp16 matrix peak, the type the products execute in: three fp16 "
                                       "MFMA products (hi x hi, hi x lo, lo x hi) per FP32-class term",
                         "fp32_class_tflops": round(tflops_d, 2),
                         "frac_of_fp32_matrix_peak": round(tflops_d / FP32_MFMA_PEAK_TFLOPS, 4),
                         "traffic": None, "algorithmic_flops_per_launch": terms * FLOPS_PER_TERM,
                         "kernel": "rmd::synth_kernel (timed with rmd::geometry_kernel and rmd::reduce_kernel: "
                                   "one IF cube)",
                         "kernel_ms_avg": round(ms_d, 3)}},
        "spread_speedup_over_direct": round(ms_d / ms, 3),
    }
    if cpu:
        from oracle import raymeta as R
        small = sc.with_rays(cpu_rays)
        t0 = time.perf_counter()
        R.if_cube(small, chirps=[0])
        dt = time.perf_counter() - t0
        n = cpu_rays * sc.n_pairs * r.n_samples
        out["cpu_baseline"] = {"value": round(n / dt, 1), "unit": "terms/s", "cores": 1,
                               "host_cores": os.cpu_count(), "kind": "oracle",
                               "sample": f"the first {cpu_rays} rays, chirp 0, all {sc.n_pairs} pairs and "
                                         f"{r.n_samples} samples (numpy FP64, single-threaded: 1 of "
                                         f"{os.cpu_count()} host cores), {dt:.1f} s"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=256, help="grid side (256 is the benchmark workload)")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--chunk-planes", type=int, default=0)
    ap.add_argument("--steps-per-sweep", type=int, default=0,
                    help="0 automatic (single steps at 256^3), 1 single steps, 2 two-step sweeps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving sweep")
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--no-adjoint", action="store_true", help="skip the gradient measurement")
    ap.add_argument("--no-sparams", action="store_true", help="skip the S-parameter measurement")
    ap.add_argument("--no-precisions", action="store_true", help="skip the FP16-storage and FP64 configurations")
    ap.add_argument("--no-if-synthesis", action="store_true", help="skip the ray-meta-data IF measurement")
    ap.add_argument("--if-only", action="store_true",
                    help="run only the ray-meta-data IF measurement and print its JSON object")
    ap.add_argument("--if-reps", type=int, default=5)
    ap.add_argument("--precision-only", action="store_true",
                    help="run only the FP16-storage and FP64 timings and print their JSON object")
    ap.add_argument("--profile-workload", choices=("cpml256", "fp16sub"), default="cpml256",
                    help="workload of --profile-run: the 256^3 FP32 one or the 512x512x256 FP16-storage substrate")
    ap.add_argument("--profile-run", action="store_true",
                    help="counter-collection driver: a few untimed steps, then a plain device copy of "
                         "COPY_MIB MiB (the known-size kernel the HBM counters are scaled by)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; no multi-GPU path exists (use --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2305_14176_amd import workloads as W
    from paper_2305_14176_amd.solver import YeeSolver

    if args.if_only:
        print(json.dumps({"if_synthesis": if_synthesis_benchmark(reps=args.if_reps,
                                                                 cpu=not args.no_cpu_baseline)}))
        return

    if args.precision_only:
        print(json.dumps({"precision_modes": precision_benchmark()}))
        return

    wl = W.cpml_block_lattice(n=args.n, steps=args.steps)
    if args.profile_run:
        if args.profile_workload == "fp16sub":
            wl = W.fp16_substrate(steps=args.steps)
        solver = YeeSolver(wl, device="cuda:0", series_len=1000, tile_rows=args.tile_rows,
                           chunk_planes=args.chunk_planes, steps_per_sweep=args.steps_per_sweep)
        solver.step(args.steps)
        src = torch.ones(COPY_MIB << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        eb = 2 if wl.precision == "f16" else 4
        print(json.dumps({"profile_run": wl.name, "steps": args.steps, "launch": solver.launch_info(),
                          "algorithmic_bytes_per_step": algorithmic_bytes_per_step(wl, elem_bytes=eb)[0],
                          "copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4}))
        return
    solver = YeeSolver(wl, device="cuda:0", series_len=max(1000, args.steps),
                       tile_rows=args.tile_rows, chunk_planes=args.chunk_planes, steps_per_sweep=args.steps_per_sweep)
    launch = solver.launch_info()
    stream = torch.cuda.current_stream()
    solver.step(args.warmup)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall0 = time.perf_counter()
    ev0.record(stream)
    solver.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall0
    ms = ev0.elapsed_time(ev1)
    ms_per_step = ms / args.steps

    copy_gbs = copy_bandwidth()
    cells = wl.cells
    value = cells * args.steps / (ms / 1e3) / 1e6
    alg, fields_b, psi_b = algorithmic_bytes_per_step(wl)
    achieved = alg / (ms_per_step / 1e3) / 1e9
    traffic = load_traffic() if launch["steps_per_sweep"] == 1 else None

    out = {
        "metric": "Mcell-updates/s (FP32 Yee step, 256^3, CPML 10); serving p50/p99 in 'serving'",
        "value": round(value, 1),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "cells": cells, "cpml_cells": list(wl.cpml_cells),
                   "materials": "8^3-cell block lattice, eps_r~U[1,10), sigma~U[0,0.1)",
                   "probes": len(wl.probes), "dft_freqs": len(wl.freqs),
                   "tile_rows": launch["tile_rows"], "chunk_planes": launch["chunk_planes"],
                   "steps_per_sweep": launch["steps_per_sweep"],
                   "parallelism": "single GPU"},
        "hbm_gbs_algorithmic": round(achieved, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": alg,
                     "kernel": ("yee::tb_kernel (two fused steps per sweep; per step)" if launch["steps_per_sweep"] == 2
                                else "yee::step_kernel (fused H + E + CPML step)"),
                     "kernel_ms_avg": round(ms_per_step, 5),
                     "copy_gbs": round(copy_gbs, 1),
                     "frac_of_copy": round(achieved / copy_gbs, 4)},
        "wall_s_timed": round(t_wall, 4),
    }
    if not args.no_precisions:
        out["precision_modes"] = precision_benchmark()
        out["precision_modes"]["error_vs_fp64_oracle"] = precision_errors()
    if not args.no_if_synthesis:
        out["if_synthesis"] = if_synthesis_benchmark(reps=args.if_reps, cpu=not args.no_cpu_baseline)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_benchmark()
    if not args.no_sparams:
        out["sparams"] = sparams_benchmark()
    if not args.no_serving:
        del solver
        torch.cuda.empty_cache()
        out["serving"] = serving_benchmark(n_requests=args.serving_requests)
        solver = None
    if not args.no_cpu_baseline:
        del solver
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
