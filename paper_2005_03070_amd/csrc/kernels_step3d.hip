// The BiCGStab step kernel on 3-D grids (step_kernel.h): phases A and B by
// z marching, boundary actions on box tiles.
#include "step_kernel.h"

namespace tgdk {

template void launch_step_dim<3>(int, int, int, const DevProb*, const int*, int, int, hipStream_t,
                                 const DevProb*);

int step_blocks_per_cu(int inner_f32, int var, int tile_id) {
    return step_blocks_per_cu_dim<3>(inner_f32, var, tile_id);
}

}  // namespace tgdk
