"""GPU tests of the batched stepper and the continuous-batching loop.

A request's results must be the same whether it runs alone (plain
``yee_step``) or in a batch next to other requests of other sizes, admitted
and retired while it runs: the batched launch computes the same per-cell
operation, so fields and probe series are compared bitwise.  The FP64
running DFT is folded once per replay in the batch and once per call alone,
so its summation order differs: it is compared to 1e-13 relative.
"""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2305_14176_amd import workloads as W
from _helpers import oracle_from_workload, rel_l2, stored

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _requests(specs):
    from paper_2305_14176_amd.serving import Request
    out = []
    for rid, (side, steps, seed, arrival) in enumerate(specs):
        out.append(Request(W.serving_request(seed, side=side, steps=steps), arrival=arrival, rid=rid))
    return out


SPECS = [(32, 70, 101, 0.0), (48, 45, 102, 0.0), (96, 90, 103, 0.0), (64, 33, 104, 0.0),
         (160, 40, 105, 0.0), (128, 52, 106, 0.0), (32, 17, 107, 0.0)]


def test_batched_results_equal_alone():
    import torch
    from paper_2305_14176_amd.serving import BatchServer, serve_one_at_a_time
    assert torch.cuda.is_available()
    keep = ("Ez", "Hx", "Ey")
    _say("[gpu] serving: alone")
    alone = {r.rid: r for r in serve_one_at_a_time(_requests(SPECS), keep_fields=keep)}
    # three slots and a budget of about two large grids (160^3 needs 216 MiB, 128^3
    # 114 MiB) force queueing and admissions mid-run
    _say("[gpu] serving: batched")
    srv = BatchServer(max_slots=3, hbm_budget=360 << 20, steps_per_replay=16, keep_fields=keep)
    mixed = {r.rid: r for r in srv.serve(_requests(SPECS))}
    assert srv.replays > 3
    assert sorted(mixed) == sorted(alone)
    for rid in alone:
        a, b = alone[rid], mixed[rid]
        np.testing.assert_array_equal(b.series, a.series, err_msg=f"series of request {rid}")
        assert rel_l2(b.dft, a.dft) <= 1e-13, (rid, rel_l2(b.dft, a.dft))
        for c in keep:
            np.testing.assert_array_equal(b.fields[c], a.fields[c], err_msg=f"{c} of request {rid}")
    srv.close()


def test_batched_streamed_replays_equal_alone():
    """Slots whose fields together exceed the last-level cache (two 160^3
    grids: 396 MB of field traffic per step) take the replay graph with
    streamed stores; with one 128^3 grid left (101 MB) the batch goes back to
    the cached graph.  Every request gives the bits it gives alone."""
    import torch
    from paper_2305_14176_amd.serving import BatchServer, serve_one_at_a_time
    assert torch.cuda.is_available()
    keep = ("Ex", "Hz")
    specs = [(160, 20, 111, 0.0), (160, 27, 112, 0.0), (128, 45, 113, 0.0)]
    _say("[gpu] serving: streamed replays, alone")
    alone = {r.rid: r for r in serve_one_at_a_time(_requests(specs), keep_fields=keep)}
    _say("[gpu] serving: streamed replays, batched")
    srv = BatchServer(max_slots=3, hbm_budget=1 << 30, steps_per_replay=8, keep_fields=keep, solo=False)
    mixed = {r.rid: r for r in srv.serve(_requests(specs))}
    assert srv.solo_runs == 0 and srv.replays > 3
    for rid in alone:
        a, b = alone[rid], mixed[rid]
        np.testing.assert_array_equal(b.series, a.series, err_msg=f"series of request {rid}")
        assert rel_l2(b.dft, a.dft) <= 1e-13, (rid, rel_l2(b.dft, a.dft))
        for c in keep:
            np.testing.assert_array_equal(b.fields[c], a.fields[c], err_msg=f"{c} of request {rid}")
    srv.close()


def test_batched_request_matches_oracle():
    from paper_2305_14176_amd.serving import BatchServer
    reqs = _requests([(48, 60, 201, 0.0), (32, 25, 202, 0.0)])
    srv = BatchServer(max_slots=4, hbm_budget=1 << 30, steps_per_replay=8, keep_fields=("Ez",))
    done = {r.rid: r for r in srv.serve(reqs)}
    for rid, req in done.items():
        sim = oracle_from_workload(req.wl)
        sim.run(req.wl.steps)
        ref = sim.series_array()
        for p in range(len(req.wl.probes)):
            assert rel_l2(req.series[:, p], ref[:, p]) <= 1e-5
            assert rel_l2(req.dft[p], sim.dft[p]) <= 1e-5
        assert rel_l2(req.fields["Ez"], stored(sim, "Ez")) <= 1e-5
    srv.close()


def test_admission_by_budget_and_slots():
    import torch
    from paper_2305_14176_amd import _lib
    from paper_2305_14176_amd.solver import YeeSolver
    lib = _lib.load()
    small = YeeSolver(W.serving_request(1, side=32, steps=10), series_len=16)
    big = YeeSolver(W.serving_request(2, side=96, steps=10), series_len=16)
    other = YeeSolver(W.serving_request(3, side=32, steps=10), series_len=16)
    b = C.c_void_p()
    assert lib.yee_batch_create(2, small.footprint + other.footprint + 4096, 8, C.byref(b)) == 0
    nb = C.c_int64()
    lib.yee_batch_footprint(2, C.byref(nb))
    t = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
    assert lib.yee_batch_bind_workspace(b, C.c_void_p((t.data_ptr() + 255) & ~255), nb.value) == 0
    slot = C.c_int32()
    assert lib.yee_batch_admit(b, big.ctx, 10, C.byref(slot)) == -6        # over budget: EAGAIN
    assert lib.yee_batch_admit(b, small.ctx, 10, C.byref(slot)) == 0
    s0 = slot.value
    assert lib.yee_batch_admit(b, small.ctx, 10, C.byref(slot)) == -1      # already admitted
    assert lib.yee_batch_admit(b, other.ctx, 10, C.byref(slot)) == 0
    third = YeeSolver(W.serving_request(4, side=32, steps=10), series_len=16)
    assert lib.yee_batch_admit(b, third.ctx, 10, C.byref(slot)) == -6      # no free slot
    act, used = C.c_int32(), C.c_int64()
    lib.yee_batch_info(b, C.byref(act), C.byref(used))
    assert act.value == 2 and used.value == small.footprint + other.footprint
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.yee_batch_run(b, stream) == 0          # 8 of 10 steps
    n = C.c_int32()
    buf = (C.c_int32 * 2)()
    lib.yee_batch_poll(b, buf, 2, C.byref(n))
    assert n.value == 0 and small.steps_done == 8
    assert lib.yee_batch_run(b, stream) == 0          # the remaining 2 steps
    lib.yee_batch_poll(b, buf, 2, C.byref(n))
    assert n.value == 2 and small.steps_done == 10 and other.steps_done == 10
    assert lib.yee_batch_release(b, s0) == 0
    assert lib.yee_batch_release(b, s0) == -4
    assert lib.yee_batch_admit(b, third.ctx, 10, C.byref(slot)) == 0
    lib.yee_batch_destroy(b)
    for s in (small, big, other, third):
        s.close()


def test_active_cell_cap_queues_and_keeps_results():
    """A cell cap smaller than two of the grids: requests wait for room (one
    larger than the cap still runs when it is alone), and every result equals
    the request run alone."""
    from paper_2305_14176_amd.serving import BatchServer, serve_one_at_a_time
    specs = [(48, 40, 301, 0.0), (64, 30, 302, 0.0), (32, 50, 303, 0.0), (96, 20, 304, 0.0)]
    keep = ("Ez",)
    _say("[gpu] serving: cell cap")
    alone = {r.rid: r for r in serve_one_at_a_time(_requests(specs), keep_fields=keep)}
    cap = 64 ** 3 + 32 ** 3        # below 96^3, and below 48^3 + 64^3 + 32^3
    srv = BatchServer(max_slots=8, hbm_budget=2 << 30, steps_per_replay=8, keep_fields=keep,
                      max_active_cells=cap)
    done = srv.serve(_requests(specs))
    by_id = {r.rid: r for r in done}
    assert sorted(by_id) == sorted(alone)
    # with the cap, the 96^3 request cannot start before the others have finished
    big = by_id[3]
    assert big.admitted >= max(by_id[i].finished for i in (0, 1, 2)) - 1e-9
    for rid, a in alone.items():
        np.testing.assert_array_equal(by_id[rid].series, a.series, err_msg=f"series of request {rid}")
        np.testing.assert_array_equal(by_id[rid].fields["Ez"], a.fields["Ez"])
    srv.close()


def test_failed_request_leaves_the_others_untouched():
    """A NaN poked into one request's initial field fails that request only
    (YEE_ENUMERIC from the health check at retirement); every other request of
    the batch equals its run alone bitwise."""
    from paper_2305_14176_amd.serving import BatchServer, serve_one_at_a_time
    specs = [(32, 40, 401, 0.0), (48, 33, 402, 0.0), (64, 37, 403, 0.0), (32, 29, 404, 0.0)]
    keep = ("Ez", "Hy")
    _say("[gpu] serving: failing request")
    alone = {r.rid: r for r in serve_one_at_a_time(_requests(specs), keep_fields=keep)}
    assert not any(r.failed for r in alone.values())
    reqs = _requests(specs)
    bad = reqs[1]
    ez = np.zeros((bad.wl.nx, bad.wl.ny, bad.wl.nz))
    ez[bad.wl.nx // 2, bad.wl.ny // 2, bad.wl.nz // 3] = np.nan
    bad.init = {"Ez": ez}
    srv = BatchServer(max_slots=4, hbm_budget=1 << 30, steps_per_replay=8, keep_fields=keep)
    done = {r.rid: r for r in srv.serve(reqs)}
    srv.close()
    assert done[1].failed and done[1].status == -5, (done[1].status, done[1].error)
    assert "YEE_ENUMERIC" in done[1].error
    for rid in (0, 2, 3):
        b, a = done[rid], alone[rid]
        assert not b.failed, b.error
        np.testing.assert_array_equal(b.series, a.series, err_msg=f"series of request {rid}")
        assert rel_l2(b.dft, a.dft) <= 1e-13
        for c in keep:
            np.testing.assert_array_equal(b.fields[c], a.fields[c], err_msg=f"{c} of request {rid}")
    # the same request alone fails the same way
    solo = serve_one_at_a_time([_requests(specs[1:2])[0]], keep_fields=())
    assert not solo[0].failed
    poked = _requests(specs[1:2])[0]
    poked.init = {"Ez": ez}
    assert serve_one_at_a_time([poked])[0].status == -5


def test_cancel_and_deadline():
    """A request cancelled by id and one whose deadline passes are retired at a
    replay boundary (slot freed); the others finish as if alone."""
    from paper_2305_14176_amd.serving import BatchServer, serve_one_at_a_time
    specs = [(32, 60, 501, 0.0), (48, 400, 502, 0.0), (64, 400, 503, 0.0), (32, 45, 504, 0.0)]
    keep = ("Ez",)
    _say("[gpu] serving: cancel and deadline")
    alone = {r.rid: r for r in serve_one_at_a_time(_requests([specs[0], specs[3]]), keep_fields=keep)}
    reqs = _requests(specs)
    reqs[2].deadline = 0.0                       # passed at the first boundary after arrival
    srv = BatchServer(max_slots=4, hbm_budget=1 << 30, steps_per_replay=8, keep_fields=keep)
    srv.cancel(1)
    done = {r.rid: r for r in srv.serve(reqs)}
    info = (C.c_int32(), C.c_int64())
    srv.lib.yee_batch_info(srv.batch, C.byref(info[0]), C.byref(info[1]))
    assert info[0].value == 0 and info[1].value == 0           # every slot and byte released
    srv.close()
    assert done[1].cancelled and done[2].cancelled
    assert "cancelled" in done[1].error and "deadline" in done[2].error
    for rid, a in ((0, alone[0]), (3, alone[1])):
        assert not done[rid].cancelled and not done[rid].failed
        np.testing.assert_array_equal(done[rid].series, a.series)
        np.testing.assert_array_equal(done[rid].fields["Ez"], a.fields["Ez"])


def test_device_reset_requeues_from_checkpoints():
    """A simulated device reset (the batch and every in-flight context
    destroyed from the host) re-queues the running requests; each resumes from
    its last checkpoint and ends bitwise equal to its run alone."""
    from paper_2305_14176_amd.serving import BatchServer, serve_one_at_a_time
    specs = [(32, 90, 601, 0.0), (48, 75, 602, 0.0), (64, 70, 603, 0.0), (32, 20, 604, 0.0)]
    keep = ("Ez", "Hx")
    _say("[gpu] serving: device reset")
    alone = {r.rid: r for r in serve_one_at_a_time(_requests(specs), keep_fields=keep)}
    srv = BatchServer(max_slots=4, hbm_budget=1 << 30, steps_per_replay=8, keep_fields=keep, checkpoint_every=3)
    done = {r.rid: r for r in srv.serve(_requests(specs), reset_after_replays=5)}
    srv.close()
    assert srv.resets == 1
    assert sum(r.requeued for r in done.values()) >= 3      # every request longer than 40 steps was in flight
    for rid, a in alone.items():
        b = done[rid]
        assert not b.failed and not b.cancelled
        np.testing.assert_array_equal(b.series, a.series, err_msg=f"series of request {rid}")
        assert rel_l2(b.dft, a.dft) <= 1e-13
        for c in keep:
            np.testing.assert_array_equal(b.fields[c], a.fields[c], err_msg=f"{c} of request {rid}")


def _requests_prec(specs, precision):
    import dataclasses
    from paper_2305_14176_amd.serving import Request
    out = []
    for rid, (side, steps, seed, arrival) in enumerate(specs):
        wl = dataclasses.replace(W.serving_request(seed, side=side, steps=steps), precision=precision,
                                 fp16_exp=(12, 12, 12, 21, 21, 21))
        out.append(Request(wl, arrival=arrival, rid=rid))
    return out


@pytest.mark.parametrize("precision", ["f16", "f64"])
def test_batched_other_precisions_equal_alone(precision):
    """A batch of FP16-storage (two samples per lane) or FP64 contexts: each
    request bitwise equal to the same request stepped alone, with admissions
    mid-run; a request of another precision fails alone."""
    import torch
    from paper_2305_14176_amd import _lib
    from paper_2305_14176_amd.serving import BatchServer, serve_one_at_a_time
    assert torch.cuda.is_available()
    specs = [(32, 40, 301, 0.0), (96, 23, 302, 0.0), (64, 31, 303, 0.0), (48, 17, 304, 0.0), (128, 12, 305, 0.0)]
    keep = ("Ex", "Ez", "Hy")
    _say(f"[gpu] serving {precision}: alone")
    alone = {r.rid: r for r in serve_one_at_a_time(_requests_prec(specs, precision), keep_fields=keep)}
    _say(f"[gpu] serving {precision}: batched")
    srv = BatchServer(max_slots=2, hbm_budget=1 << 30, steps_per_replay=8, keep_fields=keep, precision=precision)
    reqs = _requests_prec(specs, precision)
    other = _requests_prec([(32, 9, 306, 0.0)], "f32")[0]
    other.rid = 99
    mixed = {r.rid: r for r in srv.serve(reqs + [other])}
    assert srv.replays > 3
    assert mixed[99].failed and mixed[99].status == -1, (mixed[99].status, mixed[99].error)
    for rid, a in alone.items():
        b = mixed[rid]
        assert not a.failed and not b.failed, (rid, a.error, b.error)
        np.testing.assert_array_equal(b.series, a.series, err_msg=f"series of request {rid}")
        assert rel_l2(b.dft, a.dft) <= 1e-13, (rid, rel_l2(b.dft, a.dft))
        for c in keep:
            np.testing.assert_array_equal(b.fields[c], a.fields[c], err_msg=f"{c} of request {rid}")
    # the precision is fixed once the table is bound
    assert srv.lib.yee_batch_set_precision(srv.batch, _lib.PRECISIONS["f32"]) == -4     # YEE_ESTATE
    srv.close()


def test_lone_requests_run_solo_and_match_alone():
    """Three requests start together in the batch; once the two short ones
    are done the long one runs alone with yee_step in its own launch shape
    (solo), continuing from the batch's last step.  A late request runs
    alone or joins.  Every request's results are the same bits as
    one-at-a-time."""
    from paper_2305_14176_amd.serving import BatchServer, serve_one_at_a_time
    specs = [(96, 200, 401, 0.0), (64, 24, 402, 0.0), (48, 40, 403, 0.0), (32, 30, 404, 0.05)]
    keep = ("Ez", "Hy")
    alone = {r.rid: r for r in serve_one_at_a_time(_requests(specs), keep_fields=keep)}
    srv = BatchServer(max_slots=4, hbm_budget=1 << 30, steps_per_replay=8, keep_fields=keep)
    mixed = {r.rid: r for r in srv.serve(_requests(specs))}
    _say(f"[gpu] serving solo: {srv.solo_runs} of {srv.replays} replays solo")
    assert srv.solo_runs > 0 and srv.replays > srv.solo_runs
    for rid, a in alone.items():
        b = mixed[rid]
        np.testing.assert_array_equal(b.series, a.series, err_msg=f"series of request {rid}")
        assert rel_l2(b.dft, a.dft) <= 1e-13, (rid, rel_l2(b.dft, a.dft))
        for c in keep:
            np.testing.assert_array_equal(b.fields[c], a.fields[c], err_msg=f"{c} of request {rid}")
    srv.close()
