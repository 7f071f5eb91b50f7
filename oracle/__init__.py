"""FP64 CPU oracle for Fourier-probed reference-less TM retrieval.

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and
its Python binding) may import, call, link or execute anything in this
package; only the test suite, the smoke check and the benchmark's CPU
baseline leg do. It shares no code with the GPU path.

Every function states the passage of the paper (Zhong et al., "Efficient
reference-less transmission matrix retrieval for a multimode fiber using
fast Fourier transform", arXiv 2302.13524) that it follows. The plain
definitions are written out with an explicit dense probing matrix; the
FFT form is a second evaluation of the same operator whose equality with
the dense form is itself a pinned test.

Modules:
  operators  probing matrix A (Sec. 2.2, Eq. probingmatrix), forward/adjoint
  retrieval  losses, gradient (Eq. derivative), ER projection, starts,
             L-BFGS with exact quartic line search (Alg. 1), fidelity
  defocus    angular-spectrum defocus model and phase-offset solve (Sec. 2.3)
  mlp        learned-start network in FP64 (forward, backward, loss, Adam)
  preprocess half-sampling, fiber mask and per-pixel rows of the image stack
  foci       conjugate-phase foci of the retrieved rows and their power ratio
"""
