"""MI355X-native McMg: FGMRES with a learned multi-channel multigrid
preconditioner for the Helmholtz equation (arXiv 2606.30495).

The compute path is libmcmg.so (hand-written HIP kernels for gfx950 behind
the C ABI of include/mcmg.h); this package only binds it.
"""
from ._lib import Handle, McmgError, Server, solve_batch, train_step, train_loss_grad, lib, LIB_PATH  # noqa: F401
