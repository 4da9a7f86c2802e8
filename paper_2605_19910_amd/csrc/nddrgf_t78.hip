// n-diagonal DDRGF kernels of padded block sizes 112 and 128, in a translation unit of
// their own so that the block sizes build in parallel.
#define RGFK_ND_T0 7
#define RGFK_ND_T1 8
#include "nddrgf.hip"
