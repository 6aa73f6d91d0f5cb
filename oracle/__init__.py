"""FP64 CPU oracle for the SENSE / CG / MoDL / VN hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports it, and this package never
imports the product path: the two share no code.  The only shared inputs come
from the seeded generators in ``synthetic``.

Every function is a plain, slow, readable transcription of the operation it
names, in float64 / complex128, citing the part of the paper it follows:

* ``sense``  -- the SENSE model A = P F C (Methods, Applications: the inverse
  problem and the SENSE operator), its adjoint and normal operator;
* ``cg``     -- conjugate gradients for (A^H A + lambda I) x = b and the
  derivatives of the inversion operator S^{-1} (MoDL subsection);
* ``cnn``    -- the residual convolutional denoiser D_W (MoDL subsection);
* ``modl``   -- the MoDL unrolled update (eq. update_modl) and its reverse
  mode pass;
* ``vn``     -- the variational-network stage (eq. update_vn);
* ``adam``   -- the Adam update and the MSE loss (eq. network_optimize);
* ``soft_sense`` -- SENSE with several coil-map sets (Extensions to the
  SENSE-Model);
* ``toeplitz`` -- non-Cartesian SENSE by the non-uniform DFT and its normal
  operator as a PSF convolution on a twice-padded grid (Extensions to the
  SENSE-Model);
* ``ipalm``  -- iPALM and the VarNet constraint projections (Iterative
  Training Algorithms);
* ``metrics``-- relative error and NRMSE.

Where the paper is silent, the reading taken is stated in each docstring.
"""
from . import sense, cg, cnn, modl, vn, adam, metrics  # noqa: F401
