// Persistent batched kernel (defined with the sweep chain in rgf_sweep.hip), compiled
// in a translation unit of its own.
#define RGFK_BATCHED_TU
#include "rgf_sweep.hip"
