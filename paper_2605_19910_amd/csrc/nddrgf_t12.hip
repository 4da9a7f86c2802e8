// n-diagonal DDRGF kernels of padded block sizes 16 and 32, in a translation unit of
// their own so that the block sizes build in parallel.
#define RGFK_ND_T0 1
#define RGFK_ND_T1 2
#include "nddrgf.hip"
