"""MI355X-native Monte Carlo for the forest-subtracted AMM integrands of QED
graphs without lepton loops (S. Volkov, arXiv:1909.08015).

The computation runs in libamm.so (HIP kernels for gfx950 behind the C ABI in
include/amm.h); `amm` is its thin Python binding."""
from .amm import Context, AmmError, lib, CALC1, CALC2  # noqa: F401
