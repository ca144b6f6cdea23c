// Search kernels for f32 rows (instantiations of search_impl.hpp).
#include "search_impl.hpp"

namespace nsg {
kfn_t pick_search_kernel_f32(int lpr, int cpl, bool full) { return pick_kernel_t<NSG_F32>(lpr, cpl, full); }
}  // namespace nsg
