// Kernels of padded block size 32 (T = 2): compiled in a translation unit of
// their own so that the block sizes build in parallel.
#define RGFK_INST_T 2
#include "rgf_sweep.hip"
#include "ddrgf.hip"
#include "nrgf_sweep.hip"
#include "adjoint.hip"
#include "rgf_split.hip"
#include "lesser.hip"
#include "leads.hip"
#include "nrgf_split.hip"
