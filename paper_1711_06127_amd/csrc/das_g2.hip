// Delay-and-sum tiles of 2 lines: the per-call kernels' instantiations.
#include "das_tile.h"

namespace usbf {

template int launch_das_g<2, false>(const int16_t*, int, const DasArgs&, float*, hipStream_t);
template int launch_das_g<2, true>(const int16_t*, int, const DasArgs&, float*, hipStream_t);

}  // namespace usbf
