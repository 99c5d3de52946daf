"""FP64 CPU oracle for the FBP-preconditioned primal-dual (APP) TV reconstruction
of Kudo, Yamazaki, Nemoto and Takaki (arXiv 1609.06041).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The HIP library never links, imports or calls it, and this package
never imports the HIP library or its Python binding.  It shares no code with
the GPU path; the two meet only in the seeded input generator
(``paper_1609_06041_amd.synth``), which holds none of the method's arithmetic.

Everything here is plain NumPy in float64, vectorised per view, written for
readability against the paper rather than speed:

* ``geometry``  - view angles, the row/column stepping decision, grid centres
* ``projector`` - ray-driven Joseph forward projection A (Sec. 2.1 system
                  matrix; the Joseph model is this implementation's reading),
                  its transpose as the literal scatter of A, and dense A
* ``filters``   - the preconditioner D as a per-view Toeplitz filter:
                  pure ramp (Eq. 32) and smoothed ramp (Eq. 24)
* ``tv``        - forward differences, divergence, the TV norm (Eq. 2) and
                  the TV prox with non-negativity (Eq. 17), solved by the
                  projected-gradient form of Chambolle's dual projection
* ``app``       - step sizes (Eq. 16, Algorithms 1 and 2) from the largest
                  eigenvalues of the preconditioned operators,
                  Algorithm 1 / 1' (low-dose) and Algorithm 2 (few-view),
                  cost (Eq. 1), partial primal-dual gap, RMSE (Eq. 34), and
                  the error-tolerant few-view problem the conclusions name
                  (||Ax - b|| <= eps) by the same APP iteration on a split
                  primal variable (x, y)
* ``comparators`` - the unpreconditioned comparators of Sec. 4: GIST for
                  Eq. 1 and Chambolle-Pock for the few-view problem (with
                  Ax = b, or with ||Ax - b|| <= eps)
* ``unrolled``  - Algorithm 1 unrolled for a fixed number of iterations as a
                  function of (b, beta, tau, sigma), and its float64
                  central-difference gradient

Pins (tests/test_oracle_*.py) tie each function to something other than
itself: closed-form chord integrals and Gaussian projections, exact column
sums at 0 and 90 degrees, the adjoint identity and an independently derived
pixel-driven transpose, quadrature of the filter integrals, the DTFT of the
taps, closed-form TV of rectangles, the TV-prox duality gap and a 1-D
reduction solved by bounded least squares, NNLS for the beta = 0 solve,
dense eigenvalues for the operator norms, and a Chambolle-Pock solve of
the same problem for the optimum.

Parity unpinned: the iterates x^k at the exact iteration counts used for
GPU parity have no printed values in the paper (its figures are missing);
they are pinned only through the limits above.
"""
from . import geometry, projector, filters, tv, app, comparators, unrolled  # noqa: F401
