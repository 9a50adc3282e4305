// All-pairs softened gravity (Sect. 2, Eq. 5) for gfx950.
//
// Persistent ragged kernel: the grid holds a few blocks per CU; each block repeatedly takes the
// next work item (one i-tile of one cluster) from a device counter.  Items are ordered largest
// cluster first, so the long items start early and the short ones fill the tail.  Each lane keeps
// K i-particles in registers; the block streams the cluster's j-records through LDS in tiles of T
// (coalesced 16/32-byte HBM/L2 loads), and every lane reads each record from LDS as a broadcast.
// The pair term uses the VALU (v_rsq_f32 / refined v_rsq_f64); there is no contraction for MFMA.
//
// FP32 families: partial sums over one LDS tile are kept in FP32 and folded into FP64 after the
// tile (FOLD), which bounds the FP32 accumulation error by the tile length; the pure-FP32 mode
// keeps one FP32 sum.  The double-single family forms each coordinate difference from hi and lo
// parts, (xj_hi - xi_hi) + (xj_lo - xi_lo), which is exact to FP32 rounding of the difference
// itself (the subtraction of the hi parts is exact for close pairs).
//
// Results of one cluster depend only on that cluster's data and the launch's (K, T), never on
// the other clusters of the batch or on which block took which item.
#include "nb_device.h"

namespace nb {

enum { NB_FP32 = 0 };

template <int FAM, int T>
struct Lds;
template <int T>
struct Lds<FAM_F32, T> {
  float4 hi[T];
};
template <int T>
struct Lds<FAM_DS, T> {
  float4 hi[T];
  float4 lo[T];
};
template <int T>
struct Lds<FAM_F64, T> {
  double4 r[T];
};

// Common epilogue: scale by G, add the galaxy field, store, optional kick.
__device__ __forceinline__ void finish_particle(const Args& a, const DevCluster& c, int cluster, long long gi,
                                                double ax, double ay, double az, bool round32, int kick) {
  ax *= a.G;
  ay *= a.G;
  az *= a.G;
  if (round32) {
    ax = (float)ax;
    ay = (float)ay;
    az = (float)az;
  }
  if (c.flags & kFlagField) {
    double ex, ey, ez;
    galaxy_accel(a.gal, a.G, a.pos[3 * gi], a.pos[3 * gi + 1], a.pos[3 * gi + 2], ex, ey, ez);
    ax += ex;
    ay += ey;
    az += ez;
    if (round32) {
      ax = (float)ax;
      ay = (float)ay;
      az = (float)az;
    }
  }
  if (a.acc) {
    a.acc[3 * gi] = ax;
    a.acc[3 * gi + 1] = ay;
    a.acc[3 * gi + 2] = az;
  }
  if (kick) {
    const double kp = a.coef ? a.coef[3 * cluster + 2] : a.kick_post;
    double* v = a.vel + 3 * gi;
    if (round32) {
      v[0] = fmaf((float)kp, (float)ax, (float)v[0]);
      v[1] = fmaf((float)kp, (float)ay, (float)v[1]);
      v[2] = fmaf((float)kp, (float)az, (float)v[2]);
    } else {
      v[0] = fma(kp, ax, v[0]);
      v[1] = fma(kp, ay, v[1]);
      v[2] = fma(kp, az, v[2]);
    }
  }
}

// Takes the next work item for the whole block; returns -1 when none is left.
__device__ __forceinline__ int next_item(const Args& a, int* s_item) {
  __syncthreads();
  if (threadIdx.x == 0) *s_item = atomicAdd(a.item_counter, 1);
  __syncthreads();
  const int it = *s_item;
  return it < a.nitems ? it : -1;
}

// ---------------------------------------------------------------------------------------------
// FP32 and double-single families
template <int FAM, int K, int T, bool FOLD, bool MASK, bool POT>
__global__ __launch_bounds__(kBlock) void k_pair32(Args a, int kick) {
  static_assert(T <= kBlock && T % 8 == 0, "tile must fit one load per thread");
  constexpr bool DS = FAM == FAM_DS;
  __shared__ Lds<FAM, T> sh;
  __shared__ int s_item;
  const int tid = threadIdx.x;
  for (int it; (it = next_item(a, &s_item)) >= 0;) {
    const PairItem item = a.items[it];
    const DevCluster c = a.cl[item.cluster];
    float xi[K], yi[K], zi[K], xl[K], yl[K], zl[K];
    float ax[K], ay[K], az[K], pt[K];
    double Ax[K], Ay[K], Az[K], Pt[K];
    int li[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      li[k] = item.i0 + tid + k * kBlock;
      const long long gi = c.off + (li[k] < c.n ? li[k] : c.n - 1);
      const float4 p = a.rec_hi[gi];
      xi[k] = p.x;
      yi[k] = p.y;
      zi[k] = p.z;
      if (DS) {
        const float4 q = a.rec_lo[gi];
        xl[k] = q.x;
        yl[k] = q.y;
        zl[k] = q.z;
      }
      ax[k] = ay[k] = az[k] = pt[k] = 0.0f;
      Ax[k] = Ay[k] = Az[k] = Pt[k] = 0.0;
    }
    const float e2 = c.eps2f;
    for (int j0 = 0; j0 < c.n; j0 += T) {
      const int cnt = min(T, c.n - j0);
      __syncthreads();
      if (tid < T) {
        if (tid < cnt) {
          sh.hi[tid] = a.rec_hi[c.off + j0 + tid];
          if constexpr (DS) sh.lo[tid] = a.rec_lo[c.off + j0 + tid];
        } else {  // zero-mass record far away: contributes exactly 0, never NaN
          sh.hi[tid] = make_float4(1e18f, 1e18f, 1e18f, 0.0f);
          if constexpr (DS) sh.lo[tid] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
      }
      __syncthreads();
      const int cnt8 = (cnt + 7) & ~7;
      for (int u = 0; u < cnt8; u += 8) {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const float4 pj = sh.hi[u + v];
          float4 pl;
          if constexpr (DS) pl = sh.lo[u + v];
#pragma unroll
          for (int k = 0; k < K; ++k) {
            float dx = pj.x - xi[k], dy = pj.y - yi[k], dz = pj.z - zi[k];
            if constexpr (DS) {
              dx += pl.x - xl[k];
              dy += pl.y - yl[k];
              dz += pl.z - zl[k];
            }
            float r2 = fmaf(dx, dx, e2);
            r2 = fmaf(dy, dy, r2);
            r2 = fmaf(dz, dz, r2);
            const float inv = __builtin_amdgcn_rsqf(r2);
            const float mi = pj.w * inv;
            float s = mi * (inv * inv);
            if (MASK) s = r2 > 0.0f ? s : 0.0f;
            ax[k] = fmaf(dx, s, ax[k]);
            ay[k] = fmaf(dy, s, ay[k]);
            az[k] = fmaf(dz, s, az[k]);
            if (POT) pt[k] += (j0 + u + v != li[k]) ? mi : 0.0f;
          }
        }
      }
      if (FOLD) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          Ax[k] += (double)ax[k];
          Ay[k] += (double)ay[k];
          Az[k] += (double)az[k];
          ax[k] = ay[k] = az[k] = 0.0f;
          if (POT) {
            Pt[k] += (double)pt[k];
            pt[k] = 0.0f;
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (li[k] >= c.n) continue;
      const long long gi = c.off + li[k];
      if (FOLD) {
        finish_particle(a, c, item.cluster, gi, Ax[k], Ay[k], Az[k], false, kick);
        if (POT && a.pot) a.pot[gi] = -a.G * Pt[k];
      } else {
        finish_particle(a, c, item.cluster, gi, (double)ax[k], (double)ay[k], (double)az[k], true, kick);
        if (POT && a.pot) a.pot[gi] = (double)(-(float)a.G * pt[k]);
      }
    }
  }
}

// ---------------------------------------------------------------------------------------------
// FP64 family
template <int K, int T, bool MASK, bool POT>
__global__ __launch_bounds__(kBlock) void k_pair64(Args a, int kick) {
  static_assert(T <= kBlock && T % 8 == 0, "tile must fit one load per thread");
  __shared__ Lds<FAM_F64, T> sh;
  __shared__ int s_item;
  const int tid = threadIdx.x;
  for (int it; (it = next_item(a, &s_item)) >= 0;) {
    const PairItem item = a.items[it];
    const DevCluster c = a.cl[item.cluster];
    double xi[K], yi[K], zi[K], ax[K], ay[K], az[K], pt[K];
    int li[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      li[k] = item.i0 + tid + k * kBlock;
      const long long gi = c.off + (li[k] < c.n ? li[k] : c.n - 1);
      const double4 p = a.rec64[gi];
      xi[k] = p.x;
      yi[k] = p.y;
      zi[k] = p.z;
      ax[k] = ay[k] = az[k] = pt[k] = 0.0;
    }
    const double e2 = c.eps2;
    for (int j0 = 0; j0 < c.n; j0 += T) {
      const int cnt = min(T, c.n - j0);
      __syncthreads();
      if (tid < T) sh.r[tid] = tid < cnt ? a.rec64[c.off + j0 + tid] : make_double4(1e150, 1e150, 1e150, 0.0);
      __syncthreads();
      const int cnt8 = (cnt + 7) & ~7;
      for (int u = 0; u < cnt8; u += 8) {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const double4 pj = sh.r[u + v];
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const double dx = pj.x - xi[k], dy = pj.y - yi[k], dz = pj.z - zi[k];
            double r2 = fma(dx, dx, e2);
            r2 = fma(dy, dy, r2);
            r2 = fma(dz, dz, r2);
            const double inv = rsqrt_f64(r2);
            const double mi = pj.w * inv;
            double s = mi * (inv * inv);
            if (MASK) s = r2 > 0.0 ? s : 0.0;
            ax[k] = fma(dx, s, ax[k]);
            ay[k] = fma(dy, s, ay[k]);
            az[k] = fma(dz, s, az[k]);
            if (POT) pt[k] += (j0 + u + v != li[k]) ? mi : 0.0;
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (li[k] >= c.n) continue;
      const long long gi = c.off + li[k];
      finish_particle(a, c, item.cluster, gi, ax[k], ay[k], az[k], false, kick);
      if (POT && a.pot) a.pot[gi] = -a.G * pt[k];
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Dispatch over the compiled-in shapes: K in {1, 2}, T in {64, 128, 256}.
typedef void (*PairFn)(Args, int);

template <int FAM, int K, int T, bool FOLD, bool MASK, bool POT>
constexpr PairFn pick() {
  if constexpr (FAM == FAM_F64) {
    if constexpr (FOLD) return k_pair64<K, T, MASK, POT>;
    else return nullptr;  // FP64 has no separate fold path
  } else if constexpr (FAM == FAM_DS && !FOLD) {
    return nullptr;  // double-single is always folded into FP64
  } else {
    return k_pair32<FAM, K, T, FOLD, MASK, POT>;
  }
}

template <int FAM, int K, int T>
PairFn select_flags(bool fold, bool mask, bool pot) {
  const int f = (fold ? 4 : 0) | (mask ? 2 : 0) | (pot ? 1 : 0);
  switch (f) {
    case 0: return pick<FAM, K, T, false, false, false>();
    case 1: return pick<FAM, K, T, false, false, true>();
    case 2: return pick<FAM, K, T, false, true, false>();
    case 3: return pick<FAM, K, T, false, true, true>();
    case 4: return pick<FAM, K, T, true, false, false>();
    case 5: return pick<FAM, K, T, true, false, true>();
    case 6: return pick<FAM, K, T, true, true, false>();
    default: return pick<FAM, K, T, true, true, true>();
  }
}

template <int FAM>
PairFn select_shape(const TileCfg& t, bool fold, bool mask, bool pot) {
  if (t.k == 1) {
    if (t.tile == 64) return select_flags<FAM, 1, 64>(fold, mask, pot);
    if (t.tile == 128) return select_flags<FAM, 1, 128>(fold, mask, pot);
    if (t.tile == 256) return select_flags<FAM, 1, 256>(fold, mask, pot);
  } else if (t.k == 2) {
    if (t.tile == 64) return select_flags<FAM, 2, 64>(fold, mask, pot);
    if (t.tile == 128) return select_flags<FAM, 2, 128>(fold, mask, pot);
    if (t.tile == 256) return select_flags<FAM, 2, 256>(fold, mask, pot);
  }
  return nullptr;
}

static int family_of(int prec) { return prec == 3 ? FAM_F64 : prec == 2 ? FAM_DS : FAM_F32; }

bool tile_supported(int family, const TileCfg& t) {
  (void)family;
  return (t.k == 1 || t.k == 2) && (t.tile == 64 || t.tile == 128 || t.tile == 256) && t.bpc >= 1 &&
         t.bpc <= 8;
}

hipError_t launch_pair(const Args& a, const TileCfg& t, int grid, bool mask, bool potmode, bool kick,
                       hipStream_t s) {
  const int fam = family_of(a.prec);
  const bool fold = a.prec != NB_FP32;  // FP64 family uses the "fold" slot
  PairFn fn = nullptr;
  if (fam == FAM_F32)
    fn = select_shape<FAM_F32>(t, fold, mask, potmode);
  else if (fam == FAM_DS)
    fn = select_shape<FAM_DS>(t, fold, mask, potmode);
  else
    fn = select_shape<FAM_F64>(t, fold, mask, potmode);
  if (!fn) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kBlock), 0, s, a, kick ? 1 : 0);
  return hipGetLastError();
}

}  // namespace nb
