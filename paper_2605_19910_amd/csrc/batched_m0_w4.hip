// Persistent batched kernel, FP64 products, 4 waves per workgroup: a
// translation unit of its own so that the variants build in parallel.
#define RGFK_BATCHED_TU
#define RGFK_BMIXED 0
#define RGFK_BNW 4
#include "rgf_sweep.hip"
