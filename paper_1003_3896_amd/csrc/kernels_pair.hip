// Launch of the persistent pair kernel (kernels in kernels_pair_{f32,ds,f64,dl}.hip).
#include "nb_internal.h"

namespace nb {

bool tile_supported(int family, const TileCfg& t) {
  const bool kw = (t.k == 1 && (t.w == 4 || t.w == 2 || (family != FAM_DL && t.w == 1))) ||
                  (t.k == 2 && (t.w == 2 || t.w == 4));
  const bool ph = t.phase == 0 || ((family == FAM_F32 || family == FAM_DS) &&
                                   ((t.k == 1 && t.w == 4 && t.tile == 256) ||
                                    (t.k == 2 && t.w == 2 && t.tile == 256) || (t.k == 2 && t.w == 4)));
  return kw && ph && (t.tile == 128 || t.tile == 256) && t.bpc >= 1 && t.bpc <= 8;
}

hipError_t launch_pair(const Args& a, const TileCfg& t, int grid, bool mask, bool potmode, bool kick,
                       hipStream_t s) {
  PairFn fn = nullptr;
  if (a.prec == 4)
    fn = pair_kernel_dl(t, true, mask, potmode);
  else if (a.prec == 3)
    fn = pair_kernel_f64(t, true, mask, potmode);
  else if (a.prec == 2)
    fn = pair_kernel_ds(t, true, mask, potmode);
  else
    fn = pair_kernel_f32(t, a.prec != 0, mask, potmode);  // pure FP32 (0) keeps one FP32 sum
  if (!fn) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kBlock), 0, s, a, kick ? 1 : 0);
  return hipGetLastError();
}

}  // namespace nb
