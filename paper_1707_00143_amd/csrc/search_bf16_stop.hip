// Search kernels for bf16 rows with the learned early stop and the feature
// capture compiled in.
#include "search_impl.hpp"

namespace nsg {
kfn_t pick_search_kernel_bf16_stop(int lpr, int cpl, int nch) { return pick_kernel_t<NSG_BF16, 1>(lpr, cpl, nch); }
}  // namespace nsg
