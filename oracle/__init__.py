"""FP64 CPU oracle for the NUFFT Radon hot path — TEST INFRASTRUCTURE ONLY.

This package is the independent reference that the HIP path is checked
against.  It is plain, slow and written to be checked by eye against the
paper (arXiv 2304.12934, tomoCAM):

* ``radon``  — the Fourier-slice Radon transform evaluated as a direct
  non-uniform DFT (Sec. 2.1, eq. "fourier_radon"; Sec. 2.2, eq.
  "fourier_sum") and its exact adjoint (Sec. 3, eq. "transpose"), plus the
  equivalent closed-form band-limited interpolator used for brute force.
* ``qggmrf`` — the q-generalised Gaussian Markov random field prior
  (Sec. 3, eqs. "reg2" and "reg3") and its gradient.
* ``mbir``   — the objective of Sec. 3 (eq. "objfn"), its gradient
  (eq. "gradient") and the accelerated-gradient-with-restart loop
  (Sec. 3, last paragraph).

It shares no code with ``paper_2304_12934_amd`` (the product): neither
imports the other.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The product path never
falls back to it.

Functions without an independent pin say "parity unpinned" in their
docstring.
"""

from . import radon, qggmrf, mbir  # noqa: F401
