"""MI355X-native mixed-precision LOBPCG (Kressner, Ma, Shao, Algorithm 3).

The numerical work runs in liblobpcg.so (hand-written HIP kernels for gfx950
behind a C-ABI, include/lobpcg.h); this package only marshals arguments.
"""
from .solver import BatchedSolver, Solver, exact_fill, gram, mixed_qr, symbolic, syev_small  # noqa: F401
