// Delay-and-sum tiles of 4 lines: the per-call kernels' instantiations.
#include "das_tile.h"

namespace usbf {

template int launch_das_g<4, false>(const int16_t*, int, const DasArgs&, float*, hipStream_t);
template int launch_das_g<4, true>(const int16_t*, int, const DasArgs&, float*, hipStream_t);

}  // namespace usbf
