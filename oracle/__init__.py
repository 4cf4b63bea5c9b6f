"""FP64 CPU oracle for the PIC/MCC + test-particle method of Trieschmann, Schmidt
and Mussenbrock, "Particle-in-Cell/Test-Particle Simulations of Technological
Plasmas: Sputtering Transport in Capacitive Radio Frequency Discharges"
(arXiv:1607.04069).

THIS PACKAGE IS TEST INFRASTRUCTURE. It is the plain, slow, obviously correct
statement of what the GPU path computes, used only by ``tests/``, by the smoke
check in ``__graft_entry__.py`` and by the ``cpu_baseline`` leg of ``bench.py``.
The product path (the HIP library and its Python binding) never imports, calls
or links anything in here, and this package never imports the product path.

Modules
-------
constants  CODATA 2018 constants and species masses.
philox     Philox4x64-10 counter-based generator (Salmon et al., SC'11) and the
           uniform / normal maps the method draws from.
xsec       analytic cross sections of the discharge and the VHS law (Eq. 8).
pic        the PIC/MCC cycle of Sec. IV.A / Fig. 4 in FP64 numpy.
tpm        the test-particle method of Sec. IV.B (sputter source, collisional
           flight with null collisions, wall sinks).

Parity status: every function is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` against closed forms, library routines or values the
paper prints; the long-run discharge statistics are the one result the paper
gives no number for (its figures are not reproducible here) and are marked
"parity unpinned" in ``pic.run_statistics``.
"""
