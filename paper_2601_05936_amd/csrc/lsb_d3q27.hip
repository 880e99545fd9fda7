// lsb_d3q27.hip -- kernel instantiations for one velocity set (all storages).
#include "driver.h"

LSB_DEFINE_OPS(ops_d3q27, LSB_D3Q27)
