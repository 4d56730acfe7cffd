// Batched multi-source kernels (stacked frontiers).
#include "rpq_internal.h"
