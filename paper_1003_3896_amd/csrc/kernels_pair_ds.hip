// Pair-kernel instantiations of the DS family (templates in pair_kernel.h).
#include "pair_kernel.h"

namespace nb {
PairFn pair_kernel_ds(const TileCfg& t, bool fold, bool mask, bool pot) {
  return pair_select<FAM_DS>(t, fold, mask, pot);
}
}  // namespace nb
