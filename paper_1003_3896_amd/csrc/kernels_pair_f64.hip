// Pair-kernel instantiations of the F64 family (templates in pair_kernel.h).
#include "pair_kernel.h"

namespace nb {
PairFn pair_kernel_f64(const TileCfg& t, bool fold, bool mask, bool pot) {
  return pair_select<FAM_F64>(t, fold, mask, pot);
}
}  // namespace nb
