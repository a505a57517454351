// SAI preconditioner build (section IV): placeholder until the batched
// least-squares kernel lands.
#include "cm_device.h"

namespace cm {
void dev_sai_build(Dev& d, const Plan& P, double e1, double e2, double e3, hipStream_t s) {
  (void)d; (void)P; (void)e1; (void)e2; (void)e3; (void)s;
  throw Error(-7, "SAI build is not available in this build");
}
}  // namespace cm
