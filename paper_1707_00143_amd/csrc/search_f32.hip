// Search kernels for f32 rows, plain (instantiations of search_impl.hpp).
#include "search_impl.hpp"

namespace nsg {
kfn_t pick_search_kernel_f32(int lpr, int cpl, int nch) { return pick_kernel_t<NSG_F32, 0>(lpr, cpl, nch); }
}  // namespace nsg
