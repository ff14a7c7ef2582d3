"""Plain FP64 CPU oracle for Tucker-compressed FMM far-fields (TEST INFRASTRUCTURE).

This package is the reference the GPU library is checked against.  It is test
infrastructure, not part of the product: only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it.  It shares no code with the
GPU library and never imports it; both sides are fed from :mod:`synth`.

Everything is NumPy in float64 / complex128, written for readability rather than
speed.  Each function cites the passage of the paper it follows:

* :mod:`oracle.geometry` -- RWG basis functions (Section II.A, eq. (2) and ref.
  [20]), the FMM-FFT box grouping (Section II.A), the spherical angular grid and
  its size rule (Section II.A).
* :mod:`oracle.farfield` -- the far-field signatures of eq. (4), with a 3-point
  triangle rule and an independent high-order rule used only by the tests.
* :mod:`oracle.hosvd` -- the truncated higher-order SVD of Section II.B, eq. (6).
* :mod:`oracle.products` -- dense aggregation (eq. (3), Fig. 2(a)) and
  disaggregation (eq. (5), Fig. 3(a)), and the Tucker-format procedures of
  Section II.C (Fig. 2(b) and Fig. 3(b)).
* :mod:`oracle.boxgrid` -- the spectra on the FMM-FFT box grid (eq. (3), eq. (5)).
* :mod:`oracle.excitation` -- plane-wave excitation vectors, the right-hand side of
  eq. (2), which the aggregation takes as its input.

Readings of passages that are silent or garbled are listed in each module.
"""
from . import geometry, farfield, hosvd, products, boxgrid, excitation  # noqa: F401
