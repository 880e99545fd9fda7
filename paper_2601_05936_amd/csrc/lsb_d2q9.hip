// lsb_d2q9.hip -- kernel instantiations for one velocity set (all storages).
#include "driver.h"

LSB_DEFINE_OPS(ops_d2q9, LSB_D2Q9)
