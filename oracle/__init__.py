"""FP64 CPU oracle for the time-reversible FDTD gradient with compressed boundary storage.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call, link or execute anything in this
package; only the tests, the smoke check and the benchmark's CPU-baseline leg
do.  It shares no code with the HIP path: both sides only read the seeded
problem descriptions in ``workloads``.

Every function is a plain, slow restatement of the method, written for
checking by eye against the paper (Mahlau, Berg, Rosenhahn, "Numerical field
optimization for enhanced efficiency in time-reversible gradient computation
of open-source GPU-accelerated FDTD simulations", arXiv 2603.24027):

  yee      -- Eq. 1 time step, textbook Yee leapfrog with convolutional PML
              (the absorbing boundary the paper names in Section 1), forward
              step and its inverse on the lossless interior (Section 1's time
              reversal; Section 2's interface slices).
  codec    -- round-to-nearest-even conversion to smaller floating-point
              formats and back (Section 2, bit-width reduction), plus the
              per-block power-of-two scale used for FP8.
  store    -- which steps are kept when subsampling every k steps, linear
              interpolation between kept steps (Section 2, Fig. 1b), storage
              bytes and the compression factor of the Fig. 3 caption.
  adjoint  -- reverse-mode gradient of the discrete loss: full-storage
              adjoint, time-reversal adjoint with (compressed) boundary
              reinjection, and central finite differences.
  metrics  -- cosine similarity (Eq. 2) and relative L2 error.

Pins (tests/test_oracle_*.py) tie each part to something other than itself:
closed-form plane-wave eigenmodes, exact discrete energy conservation,
exact reversal, the paper's worked numbers, library casts, brute force and
finite differences.  No function here is "parity unpinned".
"""

from . import yee, codec, store, adjoint, metrics  # noqa: F401
