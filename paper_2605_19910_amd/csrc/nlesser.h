// Lesser Green's function on the band after the n-diagonal sweep (nlesser.hip).
#pragma once
#include "kernels.h"

namespace rgfk {
// a: as for the block tridiagonal lesser kernel, with bands [ne][2w+1][l][b][b] and the
// n-diagonal sweep's workspace, whose chains hold 2w more bp x bp blocks after the
// sweep's own (the last-column transfer blocks).
hipError_t launch_nrgf_lesser(const LesserArgs& a, int w, hipStream_t s);
}  // namespace rgfk
