"""Plain FP64 CPU oracle for the 1D PIC hot path of the magnetar RICS pair-cascade method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) imports, links or executes anything under ``oracle/``; only the
tests, the smoke check in ``__graft_entry__`` and the CPU-baseline leg of
``bench.py`` do.  The oracle shares no code, table or constant generator with
the HIP path: it re-derives everything from the paper in numpy float64.

Modules (each function cites the passage of the paper it follows):

* ``constants``  physical constants (CODATA 2018) and the stellar radius.
* ``geometry``   dipole field line: arc length, b, mu, x = r/R*, curvature
                 radius (Appendix B.2 "Magnetic and Radiation Geometry").
* ``rics``       RICS scattering rate, drag force and photon energy
                 (Sec. 2.1-2.2, Eqs. scatteringNdot, contdrag; Appendix A.3),
                 the (log10 gamma, s) table and its bilinear lookup, and a
                 numerical line-profile quadrature of the rate integral.
* ``philox``     Philox4x32-10 counter-based generator (Salmon et al., SC'11).
* ``drag``       Strang-split drag half step: limiter, implicit midpoint with
                 Newton-Raphson, exponential damping (Sec. 3, Eq. implicit).
* ``pic``        code units, initial state, one PIC step (gather, push, RICS,
                 move, charge-conserving deposit, absorption, pair injection,
                 atmosphere, Ampere) and the moments (Gauss residual, V_c).
* ``mlp``        FP64 forward/backward/Adam of the RICS surrogate network.

Parity status of each part is listed in the module headers; a part with no
independent pin says "parity unpinned" there.
"""
