// Delay-and-sum tiles of 1 line: the per-call kernels' instantiations.
#include "das_tile.h"

namespace usbf {

template int launch_das_g<1, false>(const int16_t*, int, const DasArgs&, float*, hipStream_t);

}  // namespace usbf
