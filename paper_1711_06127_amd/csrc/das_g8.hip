// Delay-and-sum tiles of 8 lines: the per-call kernels' instantiations.
#include "das_tile.h"

namespace usbf {

template int launch_das_g<8, false>(const int16_t*, int, const DasArgs&, float*, hipStream_t);
template int launch_das_g<8, true>(const int16_t*, int, const DasArgs&, float*, hipStream_t);

}  // namespace usbf
