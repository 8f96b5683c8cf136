// Kernels of SG-WLS passes with neighbourhood radius r = 2.
#include "sgwls_device.hpp"

namespace sgwls {
SGWLS_DEFINE_LAUNCH(2)
}  // namespace sgwls
