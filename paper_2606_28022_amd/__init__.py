"""MI355X-native FMO-xTB: fragment molecular orbital energies and gradients at
the GFN1-xTB level, computed by the HIP library libfmoxtb.so (gfx950).

The Python layer only marshals arguments into the C ABI declared in
include/fmoxtb.h; every step of the computation runs in the library's kernels.
"""

from .binding import FmoXtb, FxError, lib_path, load_library  # noqa: F401
