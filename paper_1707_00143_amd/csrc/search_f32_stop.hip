// Search kernels for f32 rows with the learned early stop and the feature
// capture compiled in.
#include "search_impl.hpp"

namespace nsg {
kfn_t pick_search_kernel_f32_stop(int lpr, int cpl, int nch) { return pick_kernel_t<NSG_F32, 1>(lpr, cpl, nch); }
}  // namespace nsg
