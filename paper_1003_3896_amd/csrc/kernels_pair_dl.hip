// Pair-kernel instantiations of the local double-single family (templates in pair_kernel.h).
#include "pair_kernel.h"

namespace nb {
PairFn pair_kernel_dl(const TileCfg& t, bool fold, bool mask, bool pot) {
  return pair_select<FAM_DL>(t, fold, mask, pot);
}
}  // namespace nb
