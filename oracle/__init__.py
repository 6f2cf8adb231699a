"""Plain FP64 CPU oracle for cyclic/acyclic compact banded solves.

TEST INFRASTRUCTURE: only tests/, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library (paper_2101_02286_amd) and never imports it.

Functions whose parity is pinned, and by what (see tests/test_oracle_pins.py):
  solve_lines / solve_axis  -- dense LU (numpy.linalg.solve) on tiny n, FFT
                               circulant diagonalisation, residual bound
  stencil_axis              -- dense circulant matrix product, closed forms
  apply_axis                -- modified-wavenumber / transfer-function closed
                               forms on Fourier-mode input
  matvec_axis               -- dense matrix product
"""
from .oracle import (OracleError, apply_axis, build, matvec_axis, num_threads, solve_axis,
                     solve_lines, stencil_axis)
from . import schemes

__all__ = ["OracleError", "apply_axis", "build", "matvec_axis", "num_threads", "solve_axis",
           "solve_lines", "stencil_axis", "schemes"]
