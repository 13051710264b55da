// V-Sample instantiations for dim = 1..10 of one integrand family (one file
// per family so that the instantiations compile in parallel).
#include "vsample_impl.h"

namespace mcubes {
MCUBES_VS_TABLE(kVsMixture, MCUBES_MIXTURE)
}  // namespace mcubes
