// lsb_d3q19.hip -- kernel instantiations for one velocity set (all storages).
#include "driver.h"

LSB_DEFINE_OPS(ops_d3q19, LSB_D3Q19)
