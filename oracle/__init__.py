"""FP64 CPU oracle for the TTNO / TTNS-block eigensolver path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised NumPy implementation of what the GPU library computes, written
from the paper (Tree Tensor Network Methods for Efficient Calculation of
Molecular Vibrational Spectra, arXiv 2512.15875).  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP path (``paper_2512_15875_amd``);
the only common module is ``workloads`` (seeded inputs, no method arithmetic).

Modules
  operators  per-mode operator matrices (harmonic-oscillator basis, Hermite DVR)
  ttno       sum-of-products -> TTNO (naive automaton + SVD compression)
  ttn        tree helpers, QR gauge moves, environments, H_eff, diagonal, Gram
  linalg     Rayleigh-Ritz, MINRES, Lanczos
  solvers    ALS, variational fitting, block LOBPCG, block inverse iteration
  exact      closed forms and dense references (normal modes, Kronecker H)
  mlp        the learned-preconditioner network (forward / backward / Adam)
"""
