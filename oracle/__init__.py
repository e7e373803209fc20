"""FP64 CPU oracle for the damped-Newton Monge-Ampere solver.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU path is checked against.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product path never calls it
and shares no code with it.

Paper: Saumier, Agueh, Khouider, "An efficient numerical algorithm for the L2
optimal transport problem with applications to image processing" (2010).

Modules
-------
fd       fourth-order centred periodic differences and Simpson weights (Section 4)
interp   periodic nearest / bilinear interpolation of grid data (Section 4)
ma       residual M(u) (eq. ma2), linearisation (eq. linearmaeq), Strain's
         FFT operator (Section 4.2), GMRES(m), the damped Newton loop (eq. linma)
fd_bicg  the finite-difference linear step of Section 4.1 (nine-point matrix, the
         augmented system of its Lemma, BiCG)
stability the power method on the inverse of the linearised operator (Section 5.1)
ma3d     the same damped Newton method in three dimensions (cofactors of a 3 x 3 matrix,
         trilinear interpolation, Strain's operator with nine derived transforms)
cnn      the warm-start network (forward, backward, Adam) in FP64

Parity status per function is listed in each module header.  Every function
here is pinned by a ``-m "not gpu"`` test against a closed form, a textbook
routine, brute force, or a value the paper prints, except where a module header
says "parity unpinned".
"""

from . import cnn, fd, fd_bicg, interp, ma, ma3d  # noqa: F401
