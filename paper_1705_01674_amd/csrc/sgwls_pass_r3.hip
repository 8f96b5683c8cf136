// Kernels of SG-WLS passes with neighbourhood radius r = 3.
#include "sgwls_device.hpp"

namespace sgwls {
SGWLS_DEFINE_LAUNCH(3)
}  // namespace sgwls
