"""FP64 oracle of port voltages and scattering parameters from the probes'
running DFTs (test infrastructure: only tests, the smoke check and the
benchmark's CPU baseline use this module).

Definitions
-----------
* Port voltage: a port q is a list of probes p with weights w; its voltage
  spectrum is the weighted sum of their running DFTs,
  V_q(f) = sum_p w_p X_p(f).  With Ez probes along a line and weights equal
  to the cell length this is the discrete line integral of E.
* Two-run scattering parameters (Sheen, Ali, Abouzahra and Kong, IEEE Trans.
  Microwave Theory Tech. 38, 1990): a reference run of the uniform structure
  gives the incident wave V_q^ref at every port position; the run with the
  device gives V_q^dut.  With the source in front of port 1,
      S_11 = (V_1^dut - V_1^ref) / V_1^ref      (reflected over incident),
      S_q1 = V_q^dut / V_q^ref,  q > 1           (transmitted over the wave a
                                                  uniform structure would carry),
  each referred to its own port position.
Both are linear-algebra definitions written out directly.
"""
import numpy as np


def port_voltages(dft, port_probes, port_weights):
    """V[q, f] = sum_i port_weights[q][i] * dft[port_probes[q][i], f]."""
    dft = np.asarray(dft, dtype=np.complex128)
    out = np.zeros((len(port_probes), dft.shape[1]), dtype=np.complex128)
    for q, (ps, ws) in enumerate(zip(port_probes, port_weights)):
        for p, w in zip(ps, ws):
            out[q] += float(w) * dft[int(p)]
    return out


def two_run(v_ref, v_dut):
    """S[q, f] for the source port q = 0: S_11 = (V_1^dut - V_1^ref) / V_1^ref and
    S_q1 = V_q^dut / V_q^ref for q > 0."""
    v_ref = np.asarray(v_ref, dtype=np.complex128)
    v_dut = np.asarray(v_dut, dtype=np.complex128)
    s = v_dut / v_ref
    s[0] = (v_dut[0] - v_ref[0]) / v_ref[0]
    return s
