// Kernels of SG-WLS passes with neighbourhood radius r = 4.
#include "sgwls_device.hpp"

namespace sgwls {
SGWLS_DEFINE_LAUNCH(4)
}  // namespace sgwls
