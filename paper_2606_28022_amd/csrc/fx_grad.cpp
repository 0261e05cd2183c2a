// FMO2 analytic gradient driver (filled in by the gradient kernels).
#include "fx_host.hpp"

namespace fx {

void Ctx::gradient() { throw FxError(FX_E_UNSUPPORTED, "gradient not available in this build"); }

}  // namespace fx
