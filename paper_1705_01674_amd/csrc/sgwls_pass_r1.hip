// Kernels of SG-WLS passes with neighbourhood radius r = 1.
#include "sgwls_device.hpp"

namespace sgwls {
SGWLS_DEFINE_LAUNCH(1)
}  // namespace sgwls
