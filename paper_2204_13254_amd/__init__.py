"""MI355X-native domain-decomposed Whitney-edge Newmark solver (HIP, gfx950).

The product is libddfem.so (C ABI in include/ddfem.h); this package holds its
sources (csrc/), its build step and a thin Python binding."""
from ._lib import DD_FP32_REFINE, DD_FP64, DDError, load  # noqa: F401
