// n-diagonal DDRGF kernels of padded block sizes 48 and 64, in a translation unit of
// their own so that the block sizes build in parallel.
#define RGFK_ND_T0 3
#define RGFK_ND_T1 4
#include "nddrgf.hip"
