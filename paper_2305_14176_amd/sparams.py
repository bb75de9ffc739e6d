"""Port voltages and two-run scattering parameters from probe DFTs: a thin
binding of ``yee_sparams`` (include/yee.h).  The arithmetic runs in libyee;
this module only marshals arrays.

A port is a list of probe indices with weights (a discrete line integral of
E when the weights are cell lengths).  With the reference run of the uniform
structure and the run with the device, and the source in front of port 0:
S_00 = (V_0^dut - V_0^ref) / V_0^ref and S_q0 = V_q^dut / V_q^ref.
"""
from __future__ import annotations

import ctypes as C
from typing import Sequence, Tuple

import numpy as np

from . import _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def sparams(dft_ref: np.ndarray, dft_dut: np.ndarray, ports: Sequence[Tuple[Sequence[int], Sequence[float]]]):
    """Returns (v_ref, v_dut, s), complex [n_ports][n_freq], from the probe DFTs
    [n_probes][n_freq] of the reference run and the device run."""
    lib = _lib.load()
    ref = np.asarray(dft_ref, dtype=np.complex128)
    dut = np.asarray(dft_dut, dtype=np.complex128)
    if ref.ndim != 2 or ref.shape != dut.shape:
        raise ValueError("dft_ref and dft_dut must be [n_probes][n_freq] arrays of one shape")
    n_probes, n_freq = ref.shape
    off = np.zeros(len(ports) + 1, np.int32)
    probes, weights = [], []
    for q, (ps, ws) in enumerate(ports):
        if len(ps) != len(ws):
            raise ValueError(f"port {q}: probe and weight lists differ in length")
        probes += [int(p) for p in ps]
        weights += [float(w) for w in ws]
        off[q + 1] = len(probes)
    pp = np.asarray(probes, np.int32)
    pw = np.asarray(weights, np.float64)
    arrs = [np.ascontiguousarray(x) for x in (ref.real, ref.imag, dut.real, dut.imag)]
    outs = [np.zeros((len(ports), n_freq)) for _ in range(6)]
    i32 = C.POINTER(C.c_int32)
    _lib.check(lib.yee_sparams(n_probes, n_freq, *[_dptr(a) for a in arrs], len(ports), off.ctypes.data_as(i32),
                               pp.ctypes.data_as(i32), _dptr(pw), *[_dptr(o) for o in outs]), "yee_sparams")
    v_ref = outs[0] + 1j * outs[1]
    v_dut = outs[2] + 1j * outs[3]
    s = outs[4] + 1j * outs[5]
    return v_ref, v_dut, s
