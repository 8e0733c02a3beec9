// Planar LIDAR observation.
#include "gd_internal.h"

namespace gdk {

hipError_t launch_lidar_impl(const SimArgs &, int, hipStream_t) { return hipErrorNotSupported; }

}  // namespace gdk
