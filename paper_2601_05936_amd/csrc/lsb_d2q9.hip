// lsb_d2q9.hip -- kernel instantiations for one velocity set (all storages),
// and the reverse mode, which exists for this velocity set.
#include "adjoint_driver.h"
#include "driver.h"

LSB_DEFINE_OPS(ops_d2q9, LSB_D2Q9)

namespace lsb {
const AdjOps* adj_ops_d2q9(int storage) {
  switch (storage) {
    case LSB_F64: return AdjDriver<LSB_F64>::table();
    case LSB_F32: return AdjDriver<LSB_F32>::table();
    default: return nullptr;
  }
}
}  // namespace lsb
