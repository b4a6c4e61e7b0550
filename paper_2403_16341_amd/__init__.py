"""MI355X-native batched small-system nonlinear solver.

Solves many independent small dense systems F(u, p) = 0 in one batch with
Newton-Raphson, Newton with Armijo backtracking, or a Powell-dogleg trust
region; Jacobians come from forward-mode dual numbers and each system is
factorised by LU with partial pivoting (arXiv 2403.16341, Sec. 2 and 3.3).

The compute path is the HIP library ``_lib/libnls.so`` behind the C ABI in
``include/nls.h``; ``paper_2403_16341_amd.nls`` is the Python binding.
Nothing is loaded at import time.
"""
__all__ = ["inputs", "nls"]
