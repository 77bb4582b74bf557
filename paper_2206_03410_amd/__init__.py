"""MI355X (gfx950) library for robust non-rigid registration by accelerated
majorization-minimization.  `amm` is the binding of the C ABI (include/amm.h),
`synth` builds seeded synthetic registration problems, `autograd` wraps the
energy and its hand-written adjoint for torch."""
__version__ = "0.1.0"
