// Search kernels for e4m3 rows, plain (instantiations of search_impl.hpp).
#include "search_impl.hpp"

namespace nsg {
kfn_t pick_search_kernel_e4m3(int lpr, int cpl, int nch) { return pick_kernel_t<NSG_E4M3, 0>(lpr, cpl, nch); }
}  // namespace nsg
