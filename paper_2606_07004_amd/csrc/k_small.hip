// Small per-run reductions that are not on the streaming path.
#include "ld_kernels.h"
