"""FP64 CPU oracle for the 3-D Yee FDTD time step.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or
links anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP path (``paper_2305_14176_amd/``); both sides receive the same seeded
inputs from ``paper_2305_14176_amd.workloads``, which holds no update
arithmetic.

The paper this package accompanies (a radar ray-tracing post-processing
method: ray meta data, IF synthesis, Eqs. 1-7) defines no full-wave solver;
none of its sections contains a spatial grid, a field update or a
time-stepping scheme.  The oracle therefore writes out the textbook scheme
(Yee 1966 staggering and leapfrog; Taflove & Hagness ch. 3 lossy Ca/Cb form;
Roden & Gedney 2000 CPML).  Every point those sources leave open is an
explicit argument of :class:`oracle.yee.Simulation`.

``oracle.sparams`` combines probe DFTs into port voltages and two-run
scattering parameters (Sheen, Ali, Abouzahra and Kong 1990), pinned on FDTD
runs of a PEC waveguide against the Yee grid's own TM11 dispersion.

``oracle.raymeta`` is the oracle of the paper's own method (Section II,
Eqs. 1-7: hit update, path lengths, antenna displacement, delays, IF
synthesis, range-Doppler transform and span masks), written from the paper's
equations; its inputs come from ``paper_2305_14176_amd.rayscene``.
"""
