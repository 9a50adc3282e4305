// Pair-kernel instantiations of the F32 family (templates in pair_kernel.h).
#include "pair_kernel.h"

namespace nb {
PairFn pair_kernel_f32(const TileCfg& t, bool fold, bool mask, bool pot) {
  return pair_select<FAM_F32>(t, fold, mask, pot);
}
}  // namespace nb
