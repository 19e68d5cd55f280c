// The BiCGStab step kernel on 2-D grids (step_kernel.h), and the launch entry
// that picks the dimension.
#include "step_kernel.h"

namespace tgdk {

template void launch_step_dim<2>(int, int, int, const DevProb*, const int*, int, int, hipStream_t,
                                 const DevProb*);
extern template void launch_step_dim<3>(int, int, int, const DevProb*, const int*, int, int, hipStream_t,
                                 const DevProb*);

void launch_step(int dim, int inner_f32, int var, int tile_id, const DevProb* probs, const int* wg_prob,
                 int total_wg, int gslot, hipStream_t s, const DevProb* single) {
    if (total_wg <= 0) return;
    if (dim == 2)
        launch_step_dim<2>(inner_f32, var, tile_id, probs, wg_prob, total_wg, gslot, s, single);
    else
        launch_step_dim<3>(inner_f32, var, tile_id, probs, wg_prob, total_wg, gslot, s, single);
}

}  // namespace tgdk
