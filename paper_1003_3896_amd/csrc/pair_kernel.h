// All-pairs softened gravity (Sect. 2, Eq. 5) for gfx950: kernel templates.
//
// Persistent ragged kernel.  The grid holds a few blocks per CU; each block repeatedly takes the
// next work item (one i-tile of one cluster against one j-range of it) from a device counter.
// Items are ordered longest j-range first, so long items start early and short ones fill the
// tail, and j-range major within a cluster, so the blocks running together share sources in L2.
//
// Block = 4 wavefronts of 64 lanes.  The 4 waves form 4/W groups; the W waves of a group hold
// the same K*64 i-particles (K per lane, in registers) and split every j-tile between them, so a
// cluster of N particles keeps N/64*W waves busy (occupancy for the latency of the dependent
// FP32 chain) without any extra global traffic.  The block streams the cluster's j-records
// through LDS in tiles of T (coalesced 16/32-byte loads from HBM/L2); each wave reads its part of
// the tile as LDS broadcasts.  At the end of an item the W partial sums of a group are combined in
// LDS in a fixed order (deterministic).  The pair term runs on the VALU (v_rsq_f32, or v_rsq_f64
// refined by one third-order Newton step); the sum is not a dense contraction, so no MFMA.
//
// FP32 families keep a wave's partial sum over its part of one tile (T/W terms) in FP32 and fold
// it into FP64 after every tile; pure-FP32 mode keeps one FP32 sum.  The double-single family forms
// each coordinate difference as (xj_hi - xi_hi) + (xj_lo - xi_lo): the hi difference is exact for
// close pairs, so the difference carries FP32 relative accuracy however close the pair is.
// The local family (particles in Hilbert-curve order) centres every coordinate on the bounding box of
// the work item's i-particles; a full j-tile that lies entirely at least 3/4 of the box diagonal D
// from that centre is computed in plain FP32 on the local coordinates: rounding both coordinates to
// FP32 moves the difference by at most 2^-24 (|d| + 2 R), and the FP32 subtraction by 2^-24 |d|
// more, at most 1.5 x 2^-22 |d| in all (R = D/2 <= 2 |d|, since |d| >= 3/4 D - R), so such a term
// is as accurate as a double-single one up to a small factor; other tiles run the double-single
// loop.  In equal-mass clusters a far tile whose bounding box lies at least 3/2 D from the centre
// uses the expanded form r^2 = |x_j|^2 + |x_i|^2 - 2 x_i.x_j (one VALU instruction less per term):
// there |x_j| >= 3 |x_i|, so every one of its eight roundings is at most 2^-24 of a quantity below
// 4 (r^2 + eps^2), a relative error of at most 32 x 2^-24 in r^2 + eps^2 (a direct FP32 r^2 has
// about 5 x 2^-24).  The sort pass computes every item's frame and two bits per j-tile (far,
// expanded) beforehand, so the pair kernel decides a tile with one scalar load and stages only the
// high parts of a far tile.
//
// The results for a particle depend only on its own cluster's data and on (T, W) (in the local
// family also on K, which sets the i-tile each coordinate frame is centred on): never on the other
// clusters of the batch, on the number of blocks, or on which block took which item.
#pragma once
#include "nb_device.h"

namespace nb {

template <int FAM, int T>
struct PairLds;
template <int T>
struct PairLds<FAM_F32, T> {
  float4 hi[T];
  __device__ const float4& lo_at(int i) const { return hi[i]; }  // unused by the FP32 family
};
template <int T>
struct PairLds<FAM_DS, T> {
  float4 hi[T];
  float4 lo[T];
  __device__ const float4& lo_at(int i) const { return lo[i]; }
};
template <int T>
struct PairLds<FAM_DL, T> : PairLds<FAM_DS, T> {};
template <int T>
struct PairLds<FAM_F64, T> {
  double4 r[T];
};

// Takes the next work item for the whole block; returns -1 when none is left.
__device__ __forceinline__ int next_item(const Args& a, int* s_item) {
  __syncthreads();
  if (threadIdx.x == 0) *s_item = atomicAdd(a.item_counter, 1);
  __syncthreads();
  const int it = *s_item;
  return it < a.nitems ? it : -1;
}

// Work-item data is the same in every lane; passing it through readfirstlane lets the compiler
// keep it in scalar registers, which leaves the vector registers to the pair loop.
__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ long long wave_uniform(long long x) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(x & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
  return (long long)(((unsigned long long)(unsigned)hi << 32) | lo);
}
__device__ __forceinline__ double wave_uniform(double x) {
  return __longlong_as_double(wave_uniform(__double_as_longlong(x)));
}
__device__ __forceinline__ float wave_uniform(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ PairItem load_item(const Args& a, int it) {
  const PairItem p = a.items[it];
  return PairItem{wave_uniform(p.cluster), wave_uniform(p.i0), wave_uniform(p.js), 0};
}
__device__ __forceinline__ DevCluster load_cluster(const Args& a, int b) {
  const DevCluster c = a.cl[b];
  DevCluster u;
  u.off = wave_uniform(c.off);
  u.part_off = wave_uniform(c.part_off);
  u.n = wave_uniform(c.n);
  u.flags = wave_uniform(c.flags);
  u.eps2 = wave_uniform(c.eps2);
  u.eps2f = wave_uniform(c.eps2f);
  u.chunk0 = wave_uniform(c.chunk0);
  u.nchunks = wave_uniform(c.nchunks);
  u.split = wave_uniform(c.split);
  u.jlen = wave_uniform(c.jlen);
  u.stile0 = wave_uniform(c.stile0);
  u.nstiles = wave_uniform(c.nstiles);
  return u;
}

typedef unsigned int v4u __attribute__((ext_vector_type(4)));
// Third word of a raw (untyped) buffer descriptor on gfx9-family GPUs: 32-bit data format.
constexpr int kBufferWord3 = 0x00020000;
__device__ __forceinline__ double as_double(unsigned lo, unsigned hi) {
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One thread's share of a j-tile, fetched from the FP64 state into registers ahead of its use so
// that the global-memory latency overlaps the previous tile's arithmetic.
struct TileRaw {
  double x, y, z, m;
  bool valid;
};

// `off` is the cluster's first particle (c.off), passed on its own so that the local family can
// keep it in a scalar register; SORTED: read the sorted copy (the local family always has one).
template <int T, bool SORTED = false>
__device__ __forceinline__ TileRaw fetch_tile(const Args& a, long long off, int j, int cnt) {
  const int tid = threadIdx.x;
  TileRaw r;
  r.valid = tid < T && tid < cnt;
  if (r.valid && (SORTED || a.spos)) {
    // sorted copy: contiguous 32-byte records, read through a buffer descriptor on the tile's
    // (scalar) base address with a 32-bit per-lane offset, so no 64-bit per-lane address stays
    // live across the tile loop; the descriptor covers the tile's cnt records only
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)(a.spos + (off + j)), (short)0, cnt * 32, kBufferWord3);
    const v4u q0 = __builtin_amdgcn_raw_buffer_load_b128(rs, tid * 32, 0, 0);
    const v4u q1 = __builtin_amdgcn_raw_buffer_load_b128(rs, tid * 32 + 16, 0, 0);
    r.x = as_double(q0.x, q0.y);
    r.y = as_double(q0.z, q0.w);
    r.z = as_double(q1.x, q1.y);
    r.m = as_double(q1.z, q1.w);
  } else if (r.valid) {
    const long long g = off + j + tid;
    r.x = a.pos[3 * g];
    r.y = a.pos[3 * g + 1];
    r.z = a.pos[3 * g + 2];
    r.m = a.mass[g];
  } else {
    r.x = r.y = r.z = r.m = 0.0;
  }
  return r;
}

// Writes the fetched share into LDS as j-records (see record32/record64), padding beyond the
// cluster with zero-weight records far away, whose terms are exactly 0 and never NaN.  The weight
// is the mass, or 1 when the cluster's masses are all equal (eq: the sums leave the mass out and
// are scaled by it once at the end).
template <int FAM, int T>
__device__ __forceinline__ void store_tile(const Args& a, PairLds<FAM, T>& sh, const TileRaw& r, const double4& ref,
                                           bool eq) {
  const int tid = threadIdx.x;
  if (tid >= T) return;
  const double w = eq ? 1.0 : r.m;
  if constexpr (FAM == FAM_F64) {
    sh.r[tid] = r.valid ? make_double4(r.x, r.y, r.z, w) : make_double4(1e150, 1e150, 1e150, 0.0);
  } else {
    if (!r.valid) {
      sh.hi[tid] = make_float4(1e18f, 1e18f, 1e18f, 0.0f);
      if constexpr (FAM != FAM_F32) sh.lo[tid] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    } else if (a.prec == 0) {
      sh.hi[tid] = make_float4((float)r.x, (float)r.y, (float)r.z, (float)w);
    } else {
      const double dx = r.x - ref.x, dy = r.y - ref.y, dz = r.z - ref.z;
      const float hx = (float)dx, hy = (float)dy, hz = (float)dz;
      sh.hi[tid] = make_float4(hx, hy, hz, (float)w);
      if constexpr (FAM != FAM_F32)
        sh.lo[tid] = make_float4((float)(dx - (double)hx), (float)(dy - (double)hy), (float)(dz - (double)hz), 0.0f);
    }
  }
}

// Writes the fetched share of a full far tile of the local family: FP32 coordinates in the work
// item's frame and the weight, the same values as store_tile's high parts (no low parts needed).
template <int FAM, int T>
__device__ __forceinline__ void store_far_tile(PairLds<FAM, T>& sh, const TileRaw& r, const double4& ref, bool eq) {
  const int tid = threadIdx.x;
  if (tid >= T) return;
  sh.hi[tid] = make_float4((float)(r.x - ref.x), (float)(r.y - ref.y), (float)(r.z - ref.z), eq ? 1.0f : (float)r.m);
}

// Writes the fetched share of a full far tile of an equal-mass cluster for the expanded form of
// r^2 (xfar_tile_terms): -2 x_j in FP32 in the work item's frame (x_j rounded to FP32 first, then
// scaled exactly by -2), and |x_j|^2 + eps^2 of that rounded x_j in three FP32 FMAs.
template <int FAM, int T>
__device__ __forceinline__ void store_xfar_tile(PairLds<FAM, T>& sh, const TileRaw& r, const double4& ref,
                                                double eps2) {
  const int tid = threadIdx.x;
  if (tid >= T) return;
  const float hx = (float)(r.x - ref.x), hy = (float)(r.y - ref.y), hz = (float)(r.z - ref.z);
  const float c = fmaf(hx, hx, fmaf(hy, hy, fmaf(hz, hz, (float)eps2)));
  sh.hi[tid] = make_float4(-2.0f * hx, -2.0f * hy, -2.0f * hz, c);
}

// Combine the W per-wave FP64 partial sums of every group in LDS (fixed order) and finish.
// red: [4 waves][64*K lanes][4] doubles (ax, ay, az, pot).
template <int K, int W, bool POT>
__device__ __forceinline__ void reduce_and_finish(const Args& a, const DevCluster& c, const PairItem& item, int ibase,
                                                  const double (&Ax)[K], const double (&Ay)[K], const double (&Az)[K],
                                                  const double (&Pt)[K], double* red, bool round32, int kick) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sub = wave % W;
  if constexpr (W > 1) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double* r = red + ((size_t)wave * 64 * K + k * 64 + lane) * 4;
      r[0] = Ax[k];
      r[1] = Ay[k];
      r[2] = Az[k];
      r[3] = POT ? Pt[k] : 0.0;
    }
    __syncthreads();
  }
  double ax[K], ay[K], az[K], pt[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    ax[k] = Ax[k];
    ay[k] = Ay[k];
    az[k] = Az[k];
    pt[k] = POT ? Pt[k] : 0.0;
    if constexpr (W > 1) {
      if (sub != 0) continue;  // only the first wave of a group combines its group's partial sums
#pragma unroll
      for (int s = 1; s < W; ++s) {
        const double* r = red + ((size_t)(wave + s) * 64 * K + k * 64 + lane) * 4;
        ax[k] += r[0];
        ay[k] += r[1];
        az[k] += r[2];
        if (POT) pt[k] += r[3];
      }
    }
  }
  if (sub != 0) return;
  if (c.split > 1 || (c.flags & kFlagDefer)) {
    // one j-range of a split cluster (or the only range of a deferred one): the combine pass adds
    // the ranges in range order and finishes the particles (kernel boundaries, not device-scope
    // fences, order the two: a fence inside this persistent kernel would write back and invalidate
    // the XCD's L2)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int li = ibase + k * 64;
      if (li < c.n) a.part[c.part_off + (long long)item.js * c.n + li] = make_double4(ax[k], ay[k], az[k], pt[k]);
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int li = ibase + k * 64;
    if (li >= c.n) continue;
    const long long gi = particle_index(a, c, li);
    finish_particle<false>(a, c, item.cluster, gi, ax[k], ay[k], az[k], round32, kick);
    if (POT && a.pot) a.pot[gi] = round32 ? (double)(-(float)a.G * (float)pt[k]) : -a.G * pt[k];
  }
}

// ---------------------------------------------------------------------------------------------
// FP32 and double-single families

// One j-record against the K i-particles of this lane:
//   d = x_j - x_i (double-single: (hi_j - hi_i) + (lo_j - lo_i)),  r2 = |d|^2 + eps^2,
//   s = m_j r2^{-3/2},  a += s d,  and with POT  pot += m_j r2^{-1/2} for j != i
// (EQ: all masses of the cluster are equal, m_j is left out here and multiplied in once later).
template <bool DS, int K, bool MASK, bool POT, bool EQ>
__device__ __forceinline__ void interact32(const float4 pj, const float4 pl, const float (&xi)[K], const float (&yi)[K],
                                           const float (&zi)[K], const float (&xl)[K], const float (&yl)[K],
                                           const float (&zl)[K], float e2, float (&ax)[K], float (&ay)[K],
                                           float (&az)[K], float (&pt)[K], const int (&li)[K], int j) {
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
    const float mi = EQ ? inv : pj.w * inv;  // equal masses: m_j is applied once, after the sum
    float s = mi * (inv * inv);
    if (MASK) s = r2 > 0.0f ? s : 0.0f;
    ax[k] = fmaf(dx, s, ax[k]);
    ay[k] = fmaf(dy, s, ay[k]);
    az[k] = fmaf(dz, s, az[k]);
    if (POT) pt[k] += (j != li[k]) ? mi : 0.0f;
  }
}

// The pair terms of this wave's share [u0, u0 + TW) of one full LDS tile (T records).
template <class LDS, bool DS, int K, int TW, int T, bool MASK, bool POT, bool PH, bool EQ>
__device__ __forceinline__ void full_tile_terms(const LDS& sh, int u0, int j0, const float (&xi)[K],
                                           const float (&yi)[K], const float (&zi)[K], const float (&xl)[K],
                                           const float (&yl)[K], const float (&zl)[K], float e2, float (&ax)[K],
                                           float (&ay)[K], float (&az)[K], float (&bx)[K], float (&by)[K],
                                           float (&bz)[K], float (&pt)[K], const int (&li)[K]) {
  if (PH) {  // rsq-grouped phases
    constexpr int BJ = 8 / K;
    for (int u = u0; u < u0 + TW; u += BJ) {
      float dx[BJ][K], dy[BJ][K], dz[BJ][K], r2[BJ][K], inv[BJ][K], mj[BJ];
#pragma unroll
      for (int v = 0; v < BJ; ++v) {
        const float4 pj = sh.hi[u + v];
        const float4 pl = sh.lo_at(u + v);
        mj[v] = pj.w;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          dx[v][k] = pj.x - xi[k];
          dy[v][k] = pj.y - yi[k];
          dz[v][k] = pj.z - zi[k];
          if constexpr (DS) {
            dx[v][k] += pl.x - xl[k];
            dy[v][k] += pl.y - yl[k];
            dz[v][k] += pl.z - zl[k];
          }
          float q = fmaf(dx[v][k], dx[v][k], e2);
          q = fmaf(dy[v][k], dy[v][k], q);
          r2[v][k] = fmaf(dz[v][k], dz[v][k], q);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int v = 0; v < BJ; ++v)
#pragma unroll
        for (int k = 0; k < K; ++k) inv[v][k] = __builtin_amdgcn_rsqf(r2[v][k]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int v = 0; v < BJ; ++v)
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float sv = (EQ ? inv[v][k] : mj[v] * inv[v][k]) * (inv[v][k] * inv[v][k]);
          if (v & 1) {
            bx[k] = fmaf(dx[v][k], sv, bx[k]);
            by[k] = fmaf(dy[v][k], sv, by[k]);
            bz[k] = fmaf(dz[v][k], sv, bz[k]);
          } else {
            ax[k] = fmaf(dx[v][k], sv, ax[k]);
            ay[k] = fmaf(dy[v][k], sv, ay[k]);
            az[k] = fmaf(dz[v][k], sv, az[k]);
          }
        }
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {  // full tile: constant trip count, two accumulator sets for ILP
#pragma unroll 2
    for (int u = u0; u < u0 + TW; u += 8) {
#pragma unroll
      for (int v = 0; v < 8; ++v)
        interact32<DS, K, MASK, POT, EQ>(sh.hi[u + v], sh.lo_at(u + v), xi, yi, zi, xl, yl, zl, e2,
                                         (v & 1) ? bx : ax, (v & 1) ? by : ay, (v & 1) ? bz : az, pt, li,
                                         j0 + u + v);
    }
  }
}

// The pair terms of this wave's share of one LDS tile of store_xfar_tile records (equal masses, the
// mass left out as in full_tile_terms), with r^2 in the expanded form
//   r^2 + eps^2 = (|x_j|^2 + eps^2) + |x_i|^2 + (-2 x_j).x_i,
// three FMAs and one add instead of three differences and three FMAs, and the sums
// S = sum s_j (-2 x_j) and W = sum s_j, from which the caller forms sum s_j (x_j - x_i) =
// -S/2 - x_i W in FP64.  qi = |x_i|^2 of the FP32 x_i, rounded once.  One accumulator set: the
// other waves on the SIMD supply the parallelism (two sets measured 1.6% slower here).
template <int K, int TW, bool MASK, bool POT, class LDS>
__device__ __forceinline__ void xfar_tile_terms(const LDS& sh, int u0, int j0, const float (&xi)[K],
                                                const float (&yi)[K], const float (&zi)[K], const float (&qi)[K],
                                                float (&ax)[K], float (&ay)[K], float (&az)[K], float (&wa)[K],
                                                float (&pt)[K], const int (&li)[K]) {
#pragma unroll 2
  for (int u = u0; u < u0 + TW; u += 8) {
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const float4 pj = sh.hi[u + v];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        float q = fmaf(pj.x, xi[k], pj.w);
        q = fmaf(pj.y, yi[k], q);
        q = fmaf(pj.z, zi[k], q);
        const float r2 = q + qi[k];
        const float inv = __builtin_amdgcn_rsqf(r2);
        float s = inv * (inv * inv);
        if (MASK) s = r2 > 0.0f ? s : 0.0f;
        ax[k] = fmaf(pj.x, s, ax[k]);
        ay[k] = fmaf(pj.y, s, ay[k]);
        az[k] = fmaf(pj.z, s, az[k]);
        wa[k] += s;
        if (POT) pt[k] += (j0 + u + v != li[k]) ? inv : 0.0f;
      }
    }
  }
}

// PH: full tiles in phases of 8 pair terms (all coordinate differences and r^2, then the 8
// v_rsq_f32 back to back, then the products and sums), fenced against compiler reordering, so the
// transcendental ops of the waves sharing a SIMD can issue in pairs.
template <int FAM, int K, int W, int T, bool FOLD, bool MASK, bool POT, bool PH>
__device__ __forceinline__ void pair32_items(const Args& a, int kick) {
  static_assert(T <= kBlock && (T / W) % 8 == 0, "tile must fit one load per thread");
  constexpr bool LOC = FAM == FAM_DL;         // local centring + near/far tiles
  constexpr bool DS = FAM == FAM_DS || LOC;  // double-single records and i-particles
  // the expanded far-tile form: one i-particle per lane only (with two, its extra sums and |x_i|^2
  // push the 80-register build into spilling inside the tile loop)
  constexpr bool XF = LOC && K == 1;
  constexpr int TW = T / W;      // records per wave per tile
  __shared__ PairLds<FAM, T> sh;
  __shared__ double red[W > 1 ? 4 * 64 * K * 4 : 1];
  __shared__ int s_item;
  // the local family parks its i-particles' low parts in LDS (each lane its own slots) and reloads
  // them for near tiles only, which keeps three vector registers out of the far-tile loops; the
  // slots share the memory of `red`, which is used only after the tile loop (a barrier between)
  static_assert(!LOC || W > 1, "the local family shares red with its low-part slots");
  float4* const s_ilo = reinterpret_cast<float4*>(red);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = wave / W, sub = wave % W;
  for (int it; (it = next_item(a, &s_item)) >= 0;) {
    // (the local family keeps the work-item data in vector registers: its 80-VGPR build ran slower
    // with the extra scalar-register pressure)
    const PairItem item = LOC ? a.items[it] : load_item(a, it);
    const DevCluster c = LOC ? a.cl[item.cluster] : load_cluster(a, item.cluster);
    // the frame the coordinates are taken in: the cluster's centre of mass, or in the local family the
    // centre of the item's i-particle box (computed with the item's far-tile bits by the sort pass)
    const double4 r0 = LOC ? a.ibox[it] : a.ref[item.cluster];
    const double4 ref = make_double4(wave_uniform(r0.x), wave_uniform(r0.y), wave_uniform(r0.z), 0.0);
    const int flag0 = LOC ? wave_uniform(item.flag0) : 0;
    // != 0: every mass of the cluster equals mc
    const double mc = LOC ? a.mconst[item.cluster] : wave_uniform(a.mconst[item.cluster]);
    const bool eq = mc != 0.0;
    const int ibase = item.i0 + grp * 64 * K + lane;
    float xi[K], yi[K], zi[K], xl[K], yl[K], zl[K], qi[K];
    float ax[K], ay[K], az[K], bx[K], by[K], bz[K], pt[K], wa[K];
    double Ax[K], Ay[K], Az[K], Pt[K];
    int li[K];
    long long gidx[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      li[k] = ibase + k * 64;
      gidx[k] = particle_index(a, c, li[k] < c.n ? li[k] : c.n - 1);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const long long gi = gidx[k];
      float4 p, q;
      record32(a, gi, ref, p, q);
      xi[k] = p.x;
      yi[k] = p.y;
      zi[k] = p.z;
      if constexpr (LOC) {
        s_ilo[k * kBlock + threadIdx.x] = q;
        xl[k] = yl[k] = zl[k] = 0.0f;  // reloaded for near tiles
      } else if constexpr (DS) {
        xl[k] = q.x;
        yl[k] = q.y;
        zl[k] = q.z;
      } else {
        xl[k] = yl[k] = zl[k] = 0.0f;
      }
      qi[k] = XF ? (float)((double)xi[k] * xi[k] + (double)yi[k] * yi[k] + (double)zi[k] * zi[k]) : 0.0f;
      ax[k] = ay[k] = az[k] = bx[k] = by[k] = bz[k] = pt[k] = wa[k] = 0.0f;
      Ax[k] = Ay[k] = Az[k] = Pt[k] = 0.0;
    }
    const float e2 = c.eps2f;
    const int jb = item.js * c.jlen, je = min(c.n, jb + c.jlen);
    const long long coff = LOC ? wave_uniform(c.off) : c.off;
    TileRaw raw = fetch_tile<T, LOC>(a, coff, jb, min(T, je - jb));
    unsigned fw = 0;  // LOC: the far-tile bits of tiles [16 q, 16 q + 16) of this item
    for (int j0 = jb; j0 < je; j0 += T) {
      const int cnt = min(T, je - j0);
      bool far = false, xfar = false;
      if constexpr (LOC) {
        // far tile: every source at least 3/4 of the item box diagonal from its centre, so the FP32
        // difference of the local coordinates is within 1.5 x 2^-22 relative of the exact one;
        // xfar: the tile's box at least 3/2 of the diagonal away, which the expanded form of r^2
        // needs in equal-mass clusters (bits computed by the sort pass; the same for the block)
        const int t = (j0 - jb) / T;
        if ((t & 15) == 0) fw = a.farflags[flag0 + (t >> 4)];
        far = (fw >> (2 * (t & 15))) & 1u;
        xfar = XF && eq && ((fw >> (2 * (t & 15) + 1)) & 1u);
      }
      __syncthreads();
      if constexpr (LOC) {
        if (xfar)
          store_xfar_tile<FAM, T>(sh, raw, ref, c.eps2);
        else if (far)
          store_far_tile<FAM, T>(sh, raw, ref, eq);
        else
          store_tile<FAM, T>(a, sh, raw, ref, eq);
      } else {
        store_tile<FAM, T>(a, sh, raw, ref, eq);
      }
      __syncthreads();
      if (j0 + T < je) raw = fetch_tile<T, LOC>(a, coff, j0 + T, min(T, je - j0 - T));
      const int u0 = sub * TW;
      if constexpr (LOC) {
        if (xfar) {
          xfar_tile_terms<K, TW, MASK, POT>(sh, u0, j0, xi, yi, zi, qi, ax, ay, az, wa, pt, li);
          // sum s_j (x_j - x_i) = -(sum s_j (-2 x_j)) / 2 - x_i sum s_j, in FP64
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const double w = (double)wa[k];
            Ax[k] += -0.5 * (double)ax[k] - (double)xi[k] * w;
            Ay[k] += -0.5 * (double)ay[k] - (double)yi[k] * w;
            Az[k] += -0.5 * (double)az[k] - (double)zi[k] * w;
            ax[k] = ay[k] = az[k] = wa[k] = 0.0f;
            if (POT) {
              Pt[k] += (double)pt[k];
              pt[k] = 0.0f;
            }
          }
          continue;
        }
        if (!far) {
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const float4 q = s_ilo[k * kBlock + threadIdx.x];
            xl[k] = q.x;
            yl[k] = q.y;
            zl[k] = q.z;
          }
        }
      }
      if (LOC && far && eq)
        full_tile_terms<PairLds<FAM, T>, false, K, TW, T, MASK, POT, false, true>(
            sh, u0, j0, xi, yi, zi, xl, yl, zl, e2, ax, ay, az, bx, by, bz, pt, li);
      else if (LOC && far)
        full_tile_terms<PairLds<FAM, T>, false, K, TW, T, MASK, POT, false, false>(
            sh, u0, j0, xi, yi, zi, xl, yl, zl, e2, ax, ay, az, bx, by, bz, pt, li);
      else if (cnt == T && eq)
        full_tile_terms<PairLds<FAM, T>, DS, K, TW, T, MASK, POT, PH, true>(sh, u0, j0, xi, yi, zi, xl, yl, zl, e2,
                                                                            ax, ay, az, bx, by, bz, pt, li);
      else if (cnt == T)
        full_tile_terms<PairLds<FAM, T>, DS, K, TW, T, MASK, POT, PH, false>(sh, u0, j0, xi, yi, zi, xl, yl, zl, e2,
                                                                             ax, ay, az, bx, by, bz, pt, li);
      else {  // partial tile: the stored weight (mass, or 1 / 0 for equal masses) zeroes the padding
        const int mine = min(TW, ((cnt - u0 + 7) & ~7));  // this wave's records, padded to 8
        for (int u = u0; u < u0 + mine; u += 8) {
#pragma unroll
          for (int v = 0; v < 8; ++v)
            interact32<DS, K, MASK, POT, false>(sh.hi[u + v], sh.lo_at(u + v), xi, yi, zi, xl, yl, zl, e2,
                                                (v & 1) ? bx : ax, (v & 1) ? by : ay, (v & 1) ? bz : az, pt, li,
                                                j0 + u + v);
        }
      }
      if (FOLD) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          Ax[k] += (double)ax[k] + (double)bx[k];
          Ay[k] += (double)ay[k] + (double)by[k];
          Az[k] += (double)az[k] + (double)bz[k];
          ax[k] = ay[k] = az[k] = 0.0f;
          bx[k] = by[k] = bz[k] = 0.0f;
          if (POT) {
            Pt[k] += (double)pt[k];
            pt[k] = 0.0f;
          }
        }
      }
    }
    if (!FOLD) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        float sx = ax[k] + bx[k], sy = ay[k] + by[k], sz = az[k] + bz[k], sp = pt[k];
        if (eq) {
          const float mf = (float)mc;
          sx *= mf;
          sy *= mf;
          sz *= mf;
          sp *= mf;
        }
        Ax[k] = sx;
        Ay[k] = sy;
        Az[k] = sz;
        Pt[k] = sp;
      }
    } else if (eq) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        Ax[k] *= mc;
        Ay[k] *= mc;
        Az[k] *= mc;
        Pt[k] *= mc;
      }
    }
    if constexpr (LOC) {
      // the cluster record again, so that its fields need not stay live (spilled) across the tiles
      int cl_index = item.cluster;
      asm volatile("" : "+v"(cl_index));
      reduce_and_finish<K, W, POT>(a, a.cl[cl_index], item, ibase, Ax, Ay, Az, Pt, red, !FOLD, kick);
    } else {
      reduce_and_finish<K, W, POT>(a, c, item, ibase, Ax, Ay, Az, Pt, red, !FOLD, kick);
    }
  }
}

template <int FAM, int K, int W, int T, bool FOLD, bool MASK, bool POT, bool PH = false>
__global__ __launch_bounds__(kBlock) void k_pair32(Args a, int kick) {
  pair32_items<FAM, K, W, T, FOLD, MASK, POT, PH>(a, kick);
}

// The local family is built for 6 waves per SIMD (at most 80 VGPRs): with both loops in one kernel
// the compiler would otherwise settle on 3, and the extra waves hide more of the FP32 chain's
// latency.  The price is a few dozen work-item set-up values spilled to scratch and reloaded once
// per tile, outside the pair loops.
template <int K, int W, int T, bool MASK, bool POT>
__global__ __launch_bounds__(kBlock, 6) void k_pair32_local(Args a, int kick) {
  pair32_items<FAM_DL, K, W, T, true, MASK, POT, false>(a, kick);
}

// ---------------------------------------------------------------------------------------------
// FP64 family

// Pair terms of records [u0, u0 + cnt) of the LDS tile (cnt a multiple of 8), FP64 throughout;
// EQ leaves the record weight out (all masses equal).
template <int K, int T, bool MASK, bool POT, bool EQ>
__device__ __forceinline__ void terms64(const PairLds<FAM_F64, T>& sh, int u0, int cnt, int j0, const double (&xi)[K],
                                        const double (&yi)[K], const double (&zi)[K], double e2, double (&ax)[K],
                                        double (&ay)[K], double (&az)[K], double (&pt)[K], const int (&li)[K]) {
  for (int u = u0; u < u0 + cnt; u += 8) {
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
        const double mi = EQ ? inv : pj.w * inv;
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

template <int K, int W, int T, bool MASK, bool POT>
__global__ __launch_bounds__(kBlock) void k_pair64(Args a, int kick) {
  static_assert(T <= kBlock && (T / W) % 8 == 0, "tile must fit one load per thread");
  constexpr int TW = T / W;
  __shared__ PairLds<FAM_F64, T> sh;
  __shared__ double red[W > 1 ? 4 * 64 * K * 4 : 1];
  __shared__ int s_item;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = wave / W, sub = wave % W;
  for (int it; (it = next_item(a, &s_item)) >= 0;) {
    const PairItem item = a.items[it];
    const DevCluster c = a.cl[item.cluster];
    const double mc = a.mconst[item.cluster];  // != 0: every mass of the cluster equals mc
    const bool eq = mc != 0.0;
    const int ibase = item.i0 + grp * 64 * K + lane;
    double xi[K], yi[K], zi[K], ax[K], ay[K], az[K], pt[K];
    int li[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      li[k] = ibase + k * 64;
      const long long gi = particle_index(a, c, li[k] < c.n ? li[k] : c.n - 1);
      const double4 p = record64(a, gi);
      xi[k] = p.x;
      yi[k] = p.y;
      zi[k] = p.z;
      ax[k] = ay[k] = az[k] = pt[k] = 0.0;
    }
    const double e2 = c.eps2;
    const int jb = item.js * c.jlen, je = min(c.n, jb + c.jlen);
    TileRaw raw = fetch_tile<T>(a, c.off, jb, min(T, je - jb));
    for (int j0 = jb; j0 < je; j0 += T) {
      const int cnt = min(T, je - j0);
      __syncthreads();
      store_tile<FAM_F64, T>(a, sh, raw, make_double4(0.0, 0.0, 0.0, 0.0), eq);
      __syncthreads();
      if (j0 + T < je) raw = fetch_tile<T>(a, c.off, j0 + T, min(T, je - j0 - T));
      const int u0 = sub * TW;
      if (cnt == T && eq)
        terms64<K, T, MASK, POT, true>(sh, u0, TW, j0, xi, yi, zi, e2, ax, ay, az, pt, li);
      else  // the stored weight (mass, or 1 / 0 for equal masses) zeroes the padding
        terms64<K, T, MASK, POT, false>(sh, u0, min(TW, ((cnt - u0 + 7) & ~7)), j0, xi, yi, zi, e2, ax, ay, az, pt,
                                        li);
    }
    if (eq) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        ax[k] *= mc;
        ay[k] *= mc;
        az[k] *= mc;
        pt[k] *= mc;
      }
    }
    reduce_and_finish<K, W, POT>(a, c, item, ibase, ax, ay, az, pt, red, false, kick);
  }
}

// Kernel for one shape and flag set of a family (nullptr when not compiled in).
template <int FAM, int K, int W, int T>
PairFn pair_flags(bool fold, bool mask, bool pot) {
  if constexpr (FAM == FAM_F64) {
    if (mask) return pot ? k_pair64<K, W, T, true, true> : k_pair64<K, W, T, true, false>;
    return pot ? k_pair64<K, W, T, false, true> : k_pair64<K, W, T, false, false>;
  } else if constexpr (FAM == FAM_DL) {
    if (mask) return pot ? k_pair32_local<K, W, T, true, true> : k_pair32_local<K, W, T, true, false>;
    return pot ? k_pair32_local<K, W, T, false, true> : k_pair32_local<K, W, T, false, false>;
  } else if constexpr (FAM == FAM_DS) {
    if (mask) return pot ? k_pair32<FAM, K, W, T, true, true, true> : k_pair32<FAM, K, W, T, true, true, false>;
    return pot ? k_pair32<FAM, K, W, T, true, false, true> : k_pair32<FAM, K, W, T, true, false, false>;
  } else {
    if (fold) {
      if (mask) return pot ? k_pair32<FAM, K, W, T, true, true, true> : k_pair32<FAM, K, W, T, true, true, false>;
      return pot ? k_pair32<FAM, K, W, T, true, false, true> : k_pair32<FAM, K, W, T, true, false, false>;
    }
    if (mask) return pot ? k_pair32<FAM, K, W, T, false, true, true> : k_pair32<FAM, K, W, T, false, true, false>;
    return pot ? k_pair32<FAM, K, W, T, false, false, true> : k_pair32<FAM, K, W, T, false, false, false>;
  }
}

// Compiled-in shapes: (K, W) in {(1,1), (1,2), (1,4), (2,2), (2,4)} (all but (1,1) for the local
// family), T in {128, 256}; the rsq-phased full-tile loop for the FP32 and double-single
// families' main shapes, used for folded sums without the self mask or the potential.
template <int FAM>
PairFn pair_select(const TileCfg& t, bool fold, bool mask, bool pot) {
  if constexpr (FAM == FAM_F32 || FAM == FAM_DS) {
    if (t.phase && fold && !mask && !pot) {
#define NB_PHASED(KK, WW, TT) \
  if (t.k == KK && t.w == WW && t.tile == TT) return k_pair32<FAM, KK, WW, TT, true, false, false, true>;
      NB_PHASED(1, 4, 256)
      NB_PHASED(2, 2, 256)
      NB_PHASED(2, 4, 128)
      NB_PHASED(2, 4, 256)
#undef NB_PHASED
    }
  }
#define NB_SHAPE(KK, WW, TT) \
  if (t.k == KK && t.w == WW && t.tile == TT) return pair_flags<FAM, KK, WW, TT>(fold, mask, pot);
  if constexpr (FAM != FAM_DL) {
    NB_SHAPE(1, 1, 128)
    NB_SHAPE(1, 1, 256)
  }
  NB_SHAPE(1, 2, 128)
  NB_SHAPE(1, 2, 256)
  NB_SHAPE(1, 4, 128)
  NB_SHAPE(1, 4, 256)
  NB_SHAPE(2, 2, 128)
  NB_SHAPE(2, 2, 256)
  NB_SHAPE(2, 4, 128)
  NB_SHAPE(2, 4, 256)
#undef NB_SHAPE
  return nullptr;
}

}  // namespace nb
