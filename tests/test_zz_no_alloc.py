"""GPU test of rmd_if_cube_static, the IF cube entry point that allocates
nothing (its workspace is a static device array of the library).

Called through the C ABI, it must give the IF cube of rmd_if_cube with a
caller workspace bit for bit (same kernels, order-free fixed-point grid,
fixed-order partition sums), on two calls in a row, the second with a
smaller input (fewer rays, samples, pairs and chirps) so that it runs over
what the first call left in the shared array.  The result is also checked
against the FP64 oracle at the IF cube's tolerance.
"""
import ctypes as C
import sys

import numpy as np
import pytest

from oracle import raymeta as R
from paper_2305_14176_amd import rayscene as S

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _static_cube(RM, ds, weights, chirp0, chirp_count):
    import torch
    lib = RM.load()
    radar = RM.radar_struct(ds.radar)
    n_pairs = ds.n_pairs
    out = torch.empty((n_pairs, chirp_count, ds.radar.n_samples), dtype=torch.complex64, device=ds.device)
    w = None if weights is None else C.c_void_p(weights.data_ptr())
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    RM.check(lib.rmd_if_cube_static(C.byref(ds.desc), C.byref(radar), n_pairs, C.c_void_p(ds.pairs.data_ptr()), w,
                                    chirp0, chirp_count, C.c_void_p(out.data_ptr()), stream), "rmd_if_cube_static")
    torch.cuda.synchronize()
    return out


def _blocks_rel(got, ref):
    num = np.sqrt(np.sum(np.abs(got - ref) ** 2, axis=-1))
    den = np.sqrt(np.sum(np.abs(ref) ** 2, axis=-1))
    return num / den


def test_static_scratch_if_cube_matches_workspace_entry_point():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_14176_amd import raymeta as RM
    RM.load()
    # first call: the larger input; second call: fewer rays, pairs and samples
    # (ragged), a chirp window [1, 3)
    cases = [(dict(n_rays=6000, n_chirps=6, n_samples=512, n_tx=2, n_rx=3, seed=41), 31, 0, 6),
             (dict(n_rays=700, n_chirps=4, n_samples=200, n_tx=1, n_rx=2, seed=42), 32, 1, 2)]
    for q, (kw, wseed, chirp0, count) in enumerate(cases):
        sc = S.small_scene(**kw)
        sc.amp = S.random_amplitudes(sc, wseed)
        ds = RM.DeviceScene(sc)
        need = RM.workspace_bytes(ds, ds.n_pairs, count)
        assert need <= RM.STATIC_SCRATCH_BYTES
        _say(f"[gpu] no-alloc call {q}: rays={sc.n_rays} chirps={chirp0}+{count} samples={ds.radar.n_samples} "
             f"pairs={ds.n_pairs} workspace={need}")
        weights = torch.as_tensor(np.asarray(sc.amp, np.float32)).to(ds.device)
        got = _static_cube(RM, ds, weights, chirp0, count)
        ref = RM.Synthesizer(ds, chirp_count=count, method="spread").run(chirp0, weights).clone()
        torch.cuda.synchronize()
        assert torch.equal(got, ref), f"call {q}: static scratch and caller workspace differ"
        err = _blocks_rel(got.cpu().numpy(), R.if_cube(sc, chirps=list(range(chirp0, chirp0 + count))))
        assert err.max() <= TOL, (q, err.max())
