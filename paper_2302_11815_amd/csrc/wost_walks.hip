// The walk kernels of one dimension and one boundary form: compiled once per
// (WOST_DIM, WOST_DS) pair so that the four sets build in parallel.
#include "wost_device.hpp"

#if !defined(WOST_DIM) || !defined(WOST_DS)
#error "compile with -DWOST_DIM=2|3 -DWOST_DS=0|1"
#endif

namespace wost {
template struct WalkPart<WOST_DIM, WOST_DS != 0>;
}  // namespace wost
