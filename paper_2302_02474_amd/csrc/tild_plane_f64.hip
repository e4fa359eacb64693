// The double-precision plane kernels and their launchers (see tild_plane.hip).
#define TILD_PART_F64 1
#include "tild_plane.hip"
