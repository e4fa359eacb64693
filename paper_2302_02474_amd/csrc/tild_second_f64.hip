// The double-precision second-order plane kernels and their launchers (see
// tild_second.hip).
#define TILD_PART_F64 1
#include "tild_second.hip"
