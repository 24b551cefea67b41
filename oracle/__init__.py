"""FP64 CPU oracle for the modal-kernel / Mueller-Nystrom / per-mode-solve path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, independent
re-statement of the method of Lai and O'Neil, "An FFT-accelerated direct solver
for electromagnetic scattering from penetrable axisymmetric objects", written
from the paper (Sections 2-5 and Appendix A).  It shares no code with the GPU
library and must only be imported by ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py``.  The product path never calls it.

Modules
  special   elliptic integrals, half-odd Legendre Q recurrences, 1/rho and
            1/rho^3 azimuthal spectra (Section 4, Appendix A)
  modal     modal Green's functions and derivatives by kernel splitting and
            FFT convolution, and the direct trapezoid for separated pairs
  discretize  panels, support nodes of the near-panel rules, interpolation
  assemble  per-mode Mueller blocks (Lemma 1, N and K expansions, eq. mullerrep)
  solve     dense per-mode solves, negative modes by parity
  farfield  far-field pattern from the surface currents
"""
