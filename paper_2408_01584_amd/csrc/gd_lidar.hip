// Planar LIDAR observation.
#include "gd_internal.h"

namespace gdk {

hipError_t launch_lidar_impl(const SimArgs &, int, hipStream_t) { return hipErrorNotSupported; }

bool lidar_kernel_node(const SimArgs *, int, hipKernelNodeParams &, void **) { return false; }

}  // namespace gdk
