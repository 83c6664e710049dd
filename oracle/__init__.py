"""FP64 CPU oracle for the McMg FGMRES hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct NumPy (complex128 / float64) implementation of
what the GPU library computes, written from the paper (McMg, arXiv
2606.30495).  Only the test suite, the package's smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.  It
shares no code with the HIP library and imports nothing from it.

Modules:
  helmholtz -- medium extension into the PML, PML stretching, the 5-/7-point
               Helmholtz+PML operator (Sec. 2.1 Eq. helm, Eq. FDM_stencil;
               App. A.1.1) and its sparse assembly.
  conv      -- multi-channel 3^D convolutions: stride 1, stride 2
               (restriction), stride-2 transposed (prolongation); GELU.
  mcmg      -- the learnable setup (Alg. 1) and the V-cycle MG(r) (Alg. 2).
  krylov    -- right-preconditioned restarted FGMRES(m) and the stationary
               McMg iteration (Sec. 3.3 Eq. mcmg_iteration).
  train     -- the residual loss L_H (Eq. loss_fun) and its gradient by
               float64 reverse mode over an independent torch forward, Adam,
               LLPF level growth (Sec. llpf).
  born      -- the periodic operator, the discrete Green operator
               (Eq. discrete_symbol) and the Born-series iterations: CBS
               (Eq. cbs_eq, Eq. cbs_gamma) and Born+McMg.

Parity status per function is stated in each module header.  Readings of the
paper where it is silent are listed at the top of each module.
"""
from . import helmholtz, conv, mcmg, krylov, born  # noqa: F401
# oracle.train imports torch; it is loaded on use (import oracle.train)
