// The BiCGStab step kernel on 3-D grids (step_kernel.h): phases A and B by
// z marching, boundary actions on box tiles.
#include "step_kernel.h"

namespace tgdk {

template void launch_step_dim<3>(int, int, int, const DevProb*, const int*, int, int, hipStream_t,
                                 const DevProb*);

}  // namespace tgdk
