// n-diagonal DDRGF kernels of padded block sizes 80 and 96, in a translation unit of
// their own so that the block sizes build in parallel.
#define RGFK_ND_T0 5
#define RGFK_ND_T1 6
#include "nddrgf.hip"
