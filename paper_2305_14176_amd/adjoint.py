"""Gradient of a probe objective with respect to per-cell eps_r (binding + autograd).

J(eps_r) = sum_{n=1}^{N} sum_p y_p[n]^2 over the workload's probes, and
dJ/d eps_r for every cell of a box, both computed by ``libyee.so``: the
forward run stores checkpoints every K steps, the backward run recomputes
each segment and applies the transposed (reverse-time) step, accumulating the
gradient in FP64.  This module only marshals arguments and device memory.

Arrays use the package's (i, j, k) index order: a design over the box
[i0, i1) x [j0, j1) x [k0, k1) has shape (i1 - i0, j1 - j0, k1 - k0).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Sequence, Tuple

import numpy as np
import torch

from . import _lib
from .solver import YeeSolver
from .workloads import Workload


def _refine_axis(seg: np.ndarray, lo: int, hi: int):
    """New segment ids along one axis: one per cell inside [lo, hi), the old
    segments split at lo and hi outside.  Returns (new ids, old id of each new id)."""
    keys = [(1, c) if lo <= c < hi else ((0 if c < lo else 2), int(seg[c])) for c in range(len(seg))]
    uniq = sorted(set(keys))
    ident = {k: q for q, k in enumerate(uniq)}
    new = np.array([ident[k] for k in keys], np.int32)
    old = np.zeros(len(uniq), np.int64)
    for c, k in enumerate(keys):
        old[ident[k]] = seg[c]
    return new, old


def design_workload(wl: Workload, box: Sequence[int]) -> Tuple[Workload, np.ndarray]:
    """Copy of `wl` whose block lattice gives every cell of `box` its own block.

    Materials are unchanged.  Returns the workload and the block index of each
    box cell, shape (bx, by, bz)."""
    i0, i1, j0, j1, k0, k1 = (int(v) for v in box)
    sx, ox = _refine_axis(np.asarray(wl.seg_x), i0, i1)
    sy, oy = _refine_axis(np.asarray(wl.seg_y), j0, j1)
    sz, oz = _refine_axis(np.asarray(wl.seg_z), k0, k1)
    nsx, nsy, nsz = len(ox), len(oy), len(oz)
    old_idx = ((oz[:, None, None] * wl.nsy + oy[None, :, None]) * wl.nsx + ox[None, None, :]).ravel()
    out = dataclasses.replace(wl, seg_x=sx, seg_y=sy, seg_z=sz, nsx=nsx, nsy=nsy, nsz=nsz,
                              eps_blk=np.asarray(wl.eps_blk, np.float64)[old_idx].copy(),
                              sig_blk=np.asarray(wl.sig_blk, np.float64)[old_idx].copy())
    ii, jj, kk = np.meshgrid(sx[i0:i1], sy[j0:j1], sz[k0:k1], indexing="ij")
    return out, (kk * nsy + jj) * nsx + ii


# Device memory the default schedule may spend on kept E histories (bytes):
# a small share of a 288 GB device (the 128^3 design problem's 16 segments of
# 64 steps need 3.3 GB).
DEFAULT_HISTORY_BUDGET = 4 << 30


def history_segments_for(n_steps: int, checkpoint_every: int, box_cells: int, elem_bytes: int,
                         budget: int = DEFAULT_HISTORY_BUDGET) -> int:
    """The newest segments whose E histories fit in `budget` bytes (at least one:
    the segment the backward run starts with), each (K + 1) x 3 x box cells."""
    segments = -(-int(n_steps) // int(checkpoint_every))
    per_segment = (int(checkpoint_every) + 1) * 3 * int(box_cells) * int(elem_bytes)
    return max(1, min(segments, int(budget) // per_segment))


class AdjointRun:
    """One forward run with checkpoints and its reverse-time gradient.

    ``history_segments``: how many of the newest segments keep the E history
    of the box from the forward run (1: every other segment is recomputed from
    its checkpoint; 0: all, and the backward run recomputes nothing), for
    (K + 1) x 3 x box cells of memory per segment.  None: as many as fit in
    DEFAULT_HISTORY_BUDGET bytes, the older segments recomputed."""

    def __init__(self, solver: YeeSolver, n_steps: int, box: Sequence[int], checkpoint_every: int = 64,
                 history_segments: int = None):
        self.solver = solver
        self.lib = solver.lib
        self.box = tuple(int(v) for v in box)
        self.shape = (self.box[1] - self.box[0], self.box[3] - self.box[2], self.box[5] - self.box[4])
        self.n_steps = int(n_steps)
        b = (C.c_int32 * 6)(*self.box)
        h = C.c_void_p()
        _lib.check(self.lib.yee_adjoint_create(solver.ctx, self.n_steps, int(checkpoint_every), b, C.byref(h)),
                   "yee_adjoint_create")
        self.handle = h
        if history_segments is None:
            cells = self.shape[0] * self.shape[1] * self.shape[2]
            elem = 8 if solver.wl.precision == "f64" else 4
            history_segments = history_segments_for(self.n_steps, checkpoint_every, cells, elem)
        self.history_segments = int(history_segments)
        if history_segments != 1:
            _lib.check(self.lib.yee_adjoint_set_history(h, int(history_segments)), "yee_adjoint_set_history")
        nb = C.c_int64()
        _lib.check(self.lib.yee_adjoint_footprint(h, C.byref(nb)), "yee_adjoint_footprint")
        self.footprint = nb.value
        with torch.cuda.device(solver.device):
            self.workspace = torch.empty(self.footprint + 256, dtype=torch.uint8, device=solver.device)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        _lib.check(self.lib.yee_adjoint_bind_workspace(h, C.c_void_p(aligned), self.footprint),
                   "yee_adjoint_bind_workspace")

    def forward(self) -> float:
        """Run the N steps from the solver's step-0 state; returns J."""
        j = C.c_double()
        _lib.check(self.lib.yee_adjoint_forward(self.handle, C.byref(j), self.solver._s()), "yee_adjoint_forward")
        return j.value

    def backward(self):
        """dJ/d eps_r of the box cells as an FP64 device tensor of shape (bx, by, bz)."""
        g = torch.empty(self.shape[::-1], dtype=torch.float64, device=self.solver.device)
        _lib.check(self.lib.yee_adjoint_backward(self.handle, C.c_void_p(g.data_ptr()), self.solver._s()),
                   "yee_adjoint_backward")
        return g.permute(2, 1, 0)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.yee_adjoint_destroy(self.handle)
            self.handle = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DesignProblem:
    """A workload whose box cells carry free eps_r values (the design)."""

    def __init__(self, wl: Workload, box: Sequence[int], n_steps: int = None, checkpoint_every: int = 64,
                 device: str = "cuda:0", history_segments: int = None):
        self.wl, self.block = design_workload(wl, box)
        self.box = tuple(int(v) for v in box)
        self.n_steps = int(wl.steps if n_steps is None else n_steps)
        self.solver = YeeSolver(self.wl, device=device, series_len=self.n_steps)
        self.run = AdjointRun(self.solver, self.n_steps, self.box, checkpoint_every, history_segments)
        self.generation = 0

    @property
    def initial_design(self) -> np.ndarray:
        return np.asarray(self.wl.eps_blk)[self.block]

    def set_design(self, eps_design: np.ndarray):
        eps = np.array(self.wl.eps_blk, np.float64)
        eps[self.block] = np.asarray(eps_design, np.float64).reshape(self.block.shape)
        self.solver.set_materials(eps)
        self.solver.reset()

    def forward(self, eps_design) -> float:
        self.set_design(eps_design)
        self.generation += 1
        return self.run.forward()

    def gradient(self):
        return self.run.backward()

    def close(self):
        self.run.close()
        self.solver.close()


class YeeObjective(torch.autograd.Function):
    """J(eps_design) with d J / d eps_design from the discrete adjoint.

    ``YeeObjective.apply(eps_design, problem)``: eps_design is a tensor of
    shape (bx, by, bz); the result is a 0-d FP64 tensor on its device.  One
    forward of a problem may be outstanding at a time."""

    @staticmethod
    def forward(ctx, eps_design, problem):
        j = problem.forward(eps_design.detach().cpu().numpy())
        ctx.problem = problem
        ctx.generation = problem.generation
        ctx.out_device = eps_design.device
        ctx.out_dtype = eps_design.dtype
        return torch.tensor(j, dtype=torch.float64, device=eps_design.device)

    @staticmethod
    def backward(ctx, grad_j):
        if ctx.problem.generation != ctx.generation:
            raise RuntimeError("the design problem ran another forward since this one")
        g = ctx.problem.gradient().to(device=ctx.out_device, dtype=ctx.out_dtype)
        return grad_j.to(g.dtype) * g, None
