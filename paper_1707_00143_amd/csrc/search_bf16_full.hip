// Search kernels for bf16 rows with every option compiled in (learned stop,
// feature capture, visit recording, pool output, statistics).
#include "search_impl.hpp"

namespace nsg {
kfn_t pick_search_kernel_bf16_full(int lpr, int cpl, int nch) { return pick_kernel_t<NSG_BF16, 2>(lpr, cpl, nch); }
}  // namespace nsg
