// O(N) kernels of libnbody for gfx950: fused kick + drift + centre-of-mass partials, and the
// energy / momentum diagnostics.  All are HBM-bound; one block of kBlock threads
// handles one chunk of kChunk particles of one cluster, so per-cluster reductions never mix
// clusters.  Every reduction runs in a fixed order (bitwise reproducible).  The update's chunk
// partials are combined by a second kernel; the energy pass, which runs rarely, lets the last
// block of a cluster to finish (device-scope atomic counter) combine them and reset the counter.
#include "nb_device.h"

namespace nb {

enum { NB_FP32 = 0, NB_FP32C = 1, NB_FP32DS = 2, NB_FP64 = 3 };

// Returns true in every thread of the block that finished cluster `cl` last (after its partial
// was published by thread 0).
__device__ __forceinline__ bool last_block_of_cluster(int* counter, int nchunks) {
  __shared__ int s_last;
  __threadfence();
  if (threadIdx.x == 0) s_last = (atomicAdd(counter, 1) == nchunks - 1);
  __syncthreads();
  const bool last = s_last;
  if (last) __threadfence();
  return last;
}

// Kick (v += kick_pre a) and drift (x += drift v) of one chunk (when `update`), and the chunk's
// partial sums for its cluster's reference point ref = sum m x / sum m of the (new) positions,
// mass-uniformity flag and bounding box (combined by k_reduce: a kernel boundary rather than a
// device-scope fence orders the two, a fence would write back the XCD's L2 in every block).
// Always launched before the pair kernel, whose work counter it clears.
constexpr int kPartials = 11;
__global__ __launch_bounds__(kBlock) void k_update(Args a, int update) {
  __shared__ double sh[6][kBlock];
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.item_counter = 0;  // the pair kernel that follows starts at item 0
  const Chunk ch = a.chunks[blockIdx.x];
  const DevCluster c = a.cl[ch.cluster];
  const int t = threadIdx.x;
  const bool valid = t < ch.count;
  const long long i = c.off + ch.start + t;
  double x[3] = {0.0, 0.0, 0.0}, m = 0.0, odd = 0.0;
  if (valid) {
    m = a.mass[i];
    odd = m != a.mass[c.off] ? 1.0 : 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) x[d] = a.pos[3 * i + d];
    if (update) {
      const double kc = a.coef ? a.coef[3 * ch.cluster] : a.kick_pre;
      const double dc = a.coef ? a.coef[3 * ch.cluster + 1] : a.drift;
      double v[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) v[d] = a.vel[3 * i + d];
      if (a.prec == NB_FP32) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const float vf = fmaf((float)kc, (float)a.acc[3 * i + d], (float)v[d]);
          const float xf = fmaf((float)dc, vf, (float)x[d]);
          v[d] = vf;
          x[d] = xf;
        }
      } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          v[d] = fma(kc, a.acc[3 * i + d], v[d]);
          x[d] = fma(dc, v[d], x[d]);
        }
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        a.vel[3 * i + d] = v[d];
        a.pos[3 * i + d] = x[d];
      }
    }
  }
  double val[5] = {m * x[0], m * x[1], m * x[2], m, odd};
  double mn[3], mx[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    mn[d] = valid ? x[d] : INFINITY;
    mx[d] = valid ? x[d] : -INFINITY;
  }
  block_reduce<5>(val, sh);
  block_minmax<3>(mn, mx, sh);
  if (t == 0) {
    double* p = a.partials + (size_t)blockIdx.x * kPartials;
    for (int q = 0; q < 5; ++q) p[q] = val[q];
    for (int d = 0; d < 3; ++d) {
      p[5 + d] = mn[d];
      p[8 + d] = mx[d];
    }
  }
}

// One block per cluster: combines the chunk partials in a fixed order into the reference point,
// the common mass (mconst = the mass when all are equal, else 0) and the bounding box.
__global__ __launch_bounds__(kBlock) void k_reduce(Args a) {
  __shared__ double sh[6][kBlock];
  const DevCluster c = a.cl[blockIdx.x];
  const int t = threadIdx.x;
  double tot[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int q = t; q < c.nchunks; q += kBlock) {
    const double* p = a.partials + (size_t)(c.chunk0 + q) * kPartials;
    for (int r = 0; r < 5; ++r) tot[r] += p[r];
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], p[5 + d]);
      hi[d] = fmax(hi[d], p[8 + d]);
    }
  }
  block_reduce<5>(tot, sh);
  block_minmax<3>(lo, hi, sh);
  if (t == 0) {
    const double M = tot[3];
    a.ref[blockIdx.x] = M > 0.0 ? make_double4(tot[0] / M, tot[1] / M, tot[2] / M, M)
                                : make_double4(0.0, 0.0, 0.0, 0.0);
    a.mconst[blockIdx.x] = tot[4] == 0.0 ? a.mass[c.off] : 0.0;
    double* b = a.box + 6 * (size_t)blockIdx.x;
    for (int d = 0; d < 3; ++d) {
      b[d] = lo[d];
      b[3 + d] = hi[d];
    }
  }
}

// Diagnostics of one chunk, then per cluster in the last block.  Sums (kEnergySums):
//   0 K  1 W  2 Uext  3-5 P  6-8 L  9-11 torque  12 M  13-15 F = sum m a_int  16 sum m |a_int|
// where a_int is the internal acceleration and pot_ws the pair potential of the pass before.
// Output per cluster (kEnergyOut): K, W, Uext, E, P, L, torque, M, F, |F|, sum m |a_int|, and a
// non-finite flag.
__global__ __launch_bounds__(kBlock) void k_energy(Args a) {
  constexpr int NS = kEnergySums;
  __shared__ double sh[NS][kBlock];
  const Chunk ch = a.chunks[blockIdx.x];
  const DevCluster c = a.cl[ch.cluster];
  const int t = threadIdx.x;
  double q[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) q[k] = 0.0;
  if (t < ch.count) {
    const long long i = c.off + ch.start + t;
    const double m = a.mass[i];
    const double x = a.pos[3 * i], y = a.pos[3 * i + 1], z = a.pos[3 * i + 2];
    const double vx = a.vel[3 * i], vy = a.vel[3 * i + 1], vz = a.vel[3 * i + 2];
    const double ax = a.eacc_ws[3 * i], ay = a.eacc_ws[3 * i + 1], az = a.eacc_ws[3 * i + 2];
    q[0] = 0.5 * m * (vx * vx + vy * vy + vz * vz);
    q[1] = 0.5 * m * a.pot_ws[i];
    q[3] = m * vx;
    q[4] = m * vy;
    q[5] = m * vz;
    q[6] = m * (y * vz - z * vy);
    q[7] = m * (z * vx - x * vz);
    q[8] = m * (x * vy - y * vx);
    q[12] = m;
    q[13] = m * ax;
    q[14] = m * ay;
    q[15] = m * az;
    q[16] = m * sqrt(ax * ax + ay * ay + az * az);
    if (c.flags & kFlagField) {
      double ex, ey, ez;
      galaxy_accel<true>(a.gal, a.G, x, y, z, ex, ey, ez);
      q[2] = m * galaxy_potential(a.gal, a.G, x, y, z);
      q[9] = m * (y * ez - z * ey);
      q[10] = m * (z * ex - x * ez);
      q[11] = m * (x * ey - y * ex);
    }
  }
  block_reduce<NS>(q, sh);
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) a.epart[(size_t)blockIdx.x * NS + k] = q[k];
  }
  if (!last_block_of_cluster(&a.chunk_counter[ch.cluster], c.nchunks)) return;
  double tot[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) tot[k] = 0.0;
  for (int p = t; p < c.nchunks; p += kBlock) {
    const double* e = a.epart + (size_t)(c.chunk0 + p) * NS;
#pragma unroll
    for (int k = 0; k < NS; ++k) tot[k] += e[k];
  }
  __syncthreads();
  block_reduce<NS>(tot, sh);
  if (t == 0) {
    double* o = a.eout + (size_t)ch.cluster * kEnergyOut;
    const double K = tot[0], W = tot[1], U = tot[2];
    o[0] = K;
    o[1] = W;
    o[2] = U;
    o[3] = K + W + U;
    for (int k = 3; k < 16; ++k) o[k + 1] = tot[k];  // P, L, torque, M, F
    o[17] = sqrt(tot[13] * tot[13] + tot[14] * tot[14] + tot[15] * tot[15]);
    o[18] = tot[16];
    bool finite = true;
    for (int k = 0; k < 19; ++k) finite = finite && isfinite(o[k]);
    o[19] = finite ? 0.0 : 1.0;
    a.chunk_counter[ch.cluster] = 0;
  }
}

// Sum the partial sums of the j-ranges of split clusters in range order and finish each particle
// (scale by G, galaxy field, store, optional kick, optional potential), as the pair kernel does for
// clusters that are not split.  Pure-FP32 mode adds the ranges in FP32.
__global__ __launch_bounds__(kBlock) void k_combine(Args a, int potmode, int kick) {
  const Chunk ch = a.chunks[blockIdx.x];
  const DevCluster c = a.cl[ch.cluster];
  const int t = threadIdx.x;
  if ((c.split <= 1 && !(c.flags & kFlagDefer)) || t >= ch.count) return;
  const int li = ch.start + t;  // position in the cluster's (sorted) order
  const long long gi = particle_index(a, c, li);
  const bool r32 = a.prec == NB_FP32;
  double ax = 0.0, ay = 0.0, az = 0.0, pt = 0.0;
  float fx = 0.0f, fy = 0.0f, fz = 0.0f, fp = 0.0f;
  for (int s = 0; s < c.split; ++s) {
    const double4 p = a.part[c.part_off + (long long)s * c.n + li];
    if (r32) {
      fx += (float)p.x;
      fy += (float)p.y;
      fz += (float)p.z;
      fp += (float)p.w;
    } else {
      ax += p.x;
      ay += p.y;
      az += p.z;
      pt += p.w;
    }
  }
  if (r32) {
    ax = fx;
    ay = fy;
    az = fz;
    pt = fp;
  }
  finish_particle<true>(a, c, ch.cluster, gi, ax, ay, az, r32, kick);
  if (potmode && a.pot) a.pot[gi] = r32 ? (double)(-(float)a.G * (float)pt) : -a.G * pt;
}

hipError_t launch_combine(const Args& a, bool potmode, bool kick, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3(a.nchunks), dim3(kBlock), 0, s, a, potmode ? 1 : 0, kick ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_update(const Args& a, int B, bool update, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(a.nchunks), dim3(kBlock), 0, s, a, update ? 1 : 0);
  hipLaunchKernelGGL(k_reduce, dim3(B), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_energy(const Args& a, hipStream_t s) {
  hipLaunchKernelGGL(k_energy, dim3(a.nchunks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace nb
