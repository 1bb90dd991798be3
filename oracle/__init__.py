"""CPU oracle for the open-rectangular-cavity scattering solver (arXiv 2008.01966).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, complex128 NumPy/SciPy
restatement of what the paper's method computes.  It exists to check the GPU library
and must never be imported by it: only the test suite, the smoke entry point and the
benchmark's CPU-baseline leg may import or run anything here.  It shares no code,
tables or constants with the HIP path; the only common module is the seeded input
description in ``workloads``.

Layout of the package (each module cites the passage of the paper it restates):

* ``problem``   - sizes, mode index sets, layer nodes, TBC quadrature grid and FFT box.
* ``columns``   - the per-mode z-columns of Sections 3-4 (finite differences, interface
                   rows) as dense systems, and the same elimination vectorised over modes.
* ``incident``  - incident plane wave and the right-hand sides g1, g2.
* ``spectrum``  - Fourier transform of the truncated free-space kernel (Section 5).
* ``tbc``       - the discrete single-layer operators of the transparent boundary
                   condition (trapezoid grid + FFT convolution), dense and FFT forms.
* ``system``    - the reduced aperture system, its block preconditioner, GMRES, and the
                   brute-force full discrete system for tiny grids.
* ``fields``    - back-substitution / field synthesis and the radar cross section.
* ``solver``    - the whole path (plan + solve) with per-phase timers.

Pins (tests marked ``not gpu``) tie each function to facts fixed by the paper or by
mathematics: closed forms, brute force on tiny grids, independent quadratures.
"""
