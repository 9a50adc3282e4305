// Space-filling-curve sort of every cluster's particles for the NB_FP32DL mode (gfx950).
//
// The pair kernel of that mode centres each work item's coordinates on its own i-particles, which
// pays off only when the particles of an i-tile (and of a j-tile) lie close together; sorting
// along a Hilbert curve of the positions makes consecutive particles spatial neighbours.  The sort
// is a stable least-significant-digit radix sort of 30-bit keys (10 bits per axis, relative to the
// cluster's bounding box) in three passes of 10 bits.  Sort tiles never span clusters, so every
// cluster is sorted on its own, and the result depends only on that cluster's positions: ties
// keep the particles' own order, and no step depends on the timing of other blocks.
#include "nb_device.h"

namespace nb {

namespace {

// Spreads the low 10 bits of v so that bit b moves to bit 3b.
__device__ __forceinline__ unsigned spread3(unsigned v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Index of the cell (x, y, z) (10 bits each) along a 3-D Hilbert curve, whose consecutive cells
// are always face neighbours (a Morton order jumps), so runs of consecutive particles have small
// bounding boxes.  Skilling's transpose method (Programming the Hilbert curve, AIP Conf. Proc.
// 707, 2004): undo the excess work of the inverse Gray code level by level, Gray-encode, then
// interleave the bits (bit b of axis a goes to key bit 3b + 2 - a).
__device__ __forceinline__ unsigned hilbert3(unsigned x, unsigned y, unsigned z) {
  unsigned X[3] = {x, y, z};
  for (unsigned Q = 1u << (kRadixBits - 1); Q > 1; Q >>= 1) {
    const unsigned P = Q - 1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;  // invert the low bits
      } else {      // exchange the low bits of X[0] and X[i]
        const unsigned t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  X[1] ^= X[0];
  X[2] ^= X[1];
  unsigned t = 0;
  for (unsigned Q = 1u << (kRadixBits - 1); Q > 1; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1;
#pragma unroll
  for (int i = 0; i < 3; ++i) X[i] ^= t;
  return (spread3(X[0]) << 2) | (spread3(X[1]) << 1) | spread3(X[2]);
}

__device__ __forceinline__ unsigned cell(double x, double lo, double scale) {
  const double q = (x - lo) * scale;
  return q <= 0.0 ? 0u : q >= (double)(kRadix - 1) ? (unsigned)(kRadix - 1) : (unsigned)q;
}

// Keys of one O(N) chunk: Hilbert index of the position's cell in the cluster's box (1024 cells
// per axis), value = local index.
__global__ __launch_bounds__(kBlock) void k_keys(Args a) {
  const Chunk ch = a.chunks[blockIdx.x];
  const DevCluster c = a.cl[ch.cluster];
  const int t = threadIdx.x;
  if (t >= ch.count) return;
  const int l = ch.start + t;
  const long long g = c.off + l;
  const double* b = a.box + 6 * (size_t)ch.cluster;
  unsigned q[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double ext = b[3 + d] - b[d];
    const double scale = ext > 0.0 ? (double)kRadix / ext : 0.0;
    q[d] = cell(a.pos[3 * g + d], b[d], scale);
  }
  a.skey[0][g] = hilbert3(q[0], q[1], q[2]);
  a.sval[0][g] = l;
}

// Digit counts of one sort tile.
__global__ __launch_bounds__(kBlock) void k_rhist(Args a, int src, int shift) {
  __shared__ int h[kRadix];
  for (int d = threadIdx.x; d < kRadix; d += kBlock) h[d] = 0;
  __syncthreads();
  const Chunk st = a.stiles[blockIdx.x];
  const long long base = a.cl[st.cluster].off + st.start;
  for (int e = threadIdx.x; e < st.count; e += kBlock) atomicAdd(&h[(a.skey[src][base + e] >> shift) & (kRadix - 1)], 1);
  __syncthreads();
  int* out = a.shist + (size_t)blockIdx.x * kRadix;
  for (int d = threadIdx.x; d < kRadix; d += kBlock) out[d] = h[d];
}

// Per cluster (one block, one thread per digit): each tile's count of a digit becomes the number
// of that digit in the cluster's earlier tiles, and sbase[cluster][digit] the number of smaller
// digits in the whole cluster; their sum is the tile's first destination for the digit.
__global__ __launch_bounds__(kRadix) void k_rscan(Args a) {
  const DevCluster c = a.cl[blockIdx.x];
  const int d = threadIdx.x;
  int run = 0;
  constexpr int kBatch = 16;  // loads in flight per thread
  for (int q0 = 0; q0 < c.nstiles; q0 += kBatch) {
    int v[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) v[b] = q0 + b < c.nstiles ? a.shist[(size_t)(c.stile0 + q0 + b) * kRadix + d] : 0;
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      if (q0 + b < c.nstiles) a.shist[(size_t)(c.stile0 + q0 + b) * kRadix + d] = run;
      run += v[b];
    }
  }
  // exclusive prefix over the digits (fixed-order Hillis-Steele scan)
  __shared__ int sum[kRadix];
  sum[d] = run;
  __syncthreads();
  for (int s = 1; s < kRadix; s <<= 1) {
    const int x = d >= s ? sum[d - s] : 0;
    __syncthreads();
    sum[d] += x;
    __syncthreads();
  }
  a.sbase[(size_t)blockIdx.x * kRadix + d] = sum[d] - run;
}

// Stable scatter of one sort tile: elements are ranked in tile order, 256 per round; inside a
// wave the lanes holding the same digit are found with one ballot per digit bit, and the four
// waves take their turns on the running per-digit destinations.
__global__ __launch_bounds__(kBlock) void k_rscatter(Args a, int src, int shift) {
  __shared__ int dst[kRadix];
  const Chunk st = a.stiles[blockIdx.x];
  const long long base = a.cl[st.cluster].off;
  const int* offs = a.shist + (size_t)blockIdx.x * kRadix;
  const int* cbase = a.sbase + (size_t)st.cluster * kRadix;
  for (int d = threadIdx.x; d < kRadix; d += kBlock) dst[d] = offs[d] + cbase[d];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int r0 = 0; r0 < st.count; r0 += kBlock) {
    const int e = r0 + threadIdx.x;
    const bool valid = e < st.count;
    unsigned key = 0;
    int val = 0;
    if (valid) {
      key = a.skey[src][base + st.start + e];
      val = a.sval[src][base + st.start + e];
    }
    const int digit = (int)((key >> shift) & (kRadix - 1));
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (digit >> b) & 1;
      const unsigned long long m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & below);
    const bool leader = valid && (peers & below) == 0;
    __syncthreads();  // dst[] holds the destinations after the previous round (and waves)
    for (int w = 0; w < kBlock / 64; ++w) {
      if (wave == w && valid) {
        const int pos = dst[digit] + rank;
        a.skey[src ^ 1][base + pos] = key;
        a.sval[src ^ 1][base + pos] = val;
      }
      __syncthreads();
      if (wave == w && leader) dst[digit] += __popcll(peers);
      __syncthreads();
    }
  }
}

// The FP64 state of the sorted order, so the pair kernel streams its j-tiles contiguously.
__global__ __launch_bounds__(kBlock) void k_gather(Args a) {
  const Chunk ch = a.chunks[blockIdx.x];
  const DevCluster c = a.cl[ch.cluster];
  const int t = threadIdx.x;
  if (t >= ch.count) return;
  const long long l = c.off + ch.start + t;
  const long long g = c.off + a.sval[1][l];
  a.spos[l] = make_double4(a.pos[3 * g], a.pos[3 * g + 1], a.pos[3 * g + 2], a.mass[g]);
}

// Bounding boxes of the j-tiles of every range of every cluster (the tiles of T sorted sources the
// pair kernel stages, from the start of each range), for the far-tile test below.  One wave per box
// slot: cluster c owns slots [tbox0, tbox0 + split ceil(jlen/128)) and uses the first
// split ceil(jlen/T) of them (range js, tile t at js ceil(jlen/T) + t); the lanes split the sources.
__global__ __launch_bounds__(kBlock) void k_tileboxes(Args a, int B, int nslots) {
  const int slot = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (slot >= nslots) return;
  int lo = 0, hi = B - 1;  // the last cluster whose first slot is <= slot
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.cl[mid].tbox0 <= slot) lo = mid;
    else hi = mid - 1;
  }
  const DevCluster c = a.cl[lo];
  const int T = a.jtile;
  const int per = (c.jlen + T - 1) / T;  // tiles of a full range
  const int local = slot - c.tbox0, js = local / per, t = local % per;
  if (js >= c.split) return;
  const int jb = js * c.jlen, je = min(c.n, jb + c.jlen), j0 = jb + t * T;
  if (j0 >= je) return;
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int m = lane; m < T && j0 + m < je; m += 64) {
    const double4 p = a.spos[c.off + j0 + m];
    v[0] = fmin(v[0], p.x);
    v[1] = fmin(v[1], p.y);
    v[2] = fmin(v[2], p.z);
    v[3] = fmax(v[3], p.x);
    v[4] = fmax(v[4], p.y);
    v[5] = fmax(v[5], p.z);
  }
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      v[d] = fmin(v[d], __shfl_xor(v[d], s));
      v[3 + d] = fmax(v[3 + d], __shfl_xor(v[3 + d], s));
    }
  double* out = a.tbox + 6 * (size_t)slot;
#pragma unroll
  for (int d = 0; d < 6; ++d)
    if (lane == d) out[d] = v[d];
}

// The 16 low bits of x moved to the even bit positions 0, 2, .., 30.
__device__ __forceinline__ unsigned spread_even(unsigned x) {
  x = (x | (x << 8)) & 0x00ff00ffu;
  x = (x | (x << 4)) & 0x0f0f0f0fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}

// The local frame and the far-tile bits of the pair work items (one wave per item), from the sorted
// FP64 copy.  The frame is centred on the bounding box of the item's i-particles, ref = (lo + hi)/2,
// with far2 = (3/4 of the box diagonal D)^2 (with a 1e-6 relative margin); j-tile t of the item's
// range is far when it is full and every one of its sources lies at |x_j - ref|^2 >= far2: then the
// FP32 difference of two coordinates in that frame is within 1.5 x 2^-22 of the exact difference
// (relative), and the pair kernel computes it without the double-single correction.  A tile whose
// bounding box already lies that far (one lane per tile, 64 tiles per pass) is far; only the others
// are tested source by source (four tiles at a time, 16 lanes each, so that their loads are in
// flight together).  A far tile whose bounding box lies at least 3/2 D from the centre is also
// marked for the expanded form of r^2 (the pair kernel's xfar_tile_terms), whose rounding error
// grows as the sources come closer to the frame's centre.  Two bits per tile, 16 consecutive tiles
// per word: bit 2b far, bit 2b + 1 expanded.
__global__ __launch_bounds__(kBlock) void k_farflags(Args a) {
  const int it = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (it >= a.nitems) return;
  const PairItem item = a.items[it];
  const DevCluster c = a.cl[item.cluster];
  const int i1 = min(c.n, item.i0 + a.item_tile);
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int l = item.i0 + lane; l < i1; l += 64) {
    const double4 q = a.spos[c.off + l];
    v[0] = fmin(v[0], q.x);
    v[1] = fmin(v[1], q.y);
    v[2] = fmin(v[2], q.z);
    v[3] = fmax(v[3], q.x);
    v[4] = fmax(v[4], q.y);
    v[5] = fmax(v[5], q.z);
  }
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      v[d] = fmin(v[d], __shfl_xor(v[d], s));
      v[3 + d] = fmax(v[3 + d], __shfl_xor(v[3 + d], s));
    }
  const double dx = v[3] - v[0], dy = v[4] - v[1], dz = v[5] - v[2];
  const double rx = 0.5 * (v[0] + v[3]), ry = 0.5 * (v[1] + v[4]), rz = 0.5 * (v[2] + v[5]);
  const double diag2 = dx * dx + dy * dy + dz * dz;
  const double far2 = diag2 * (0.5625 * (1.0 + 1e-6)), farx2 = diag2 * (2.25 * (1.0 + 1e-6));
  if (lane == 0) a.ibox[it] = make_double4(rx, ry, rz, far2);
  const int T = a.jtile;
  const int jb = item.js * c.jlen, je = min(c.n, jb + c.jlen);
  const int ntiles = (je - jb + T - 1) / T, nwords = (ntiles + 15) / 16;
  const double* tb = a.tbox + 6 * ((size_t)c.tbox0 + (size_t)item.js * ((c.jlen + T - 1) / T));
  for (int q = 0; 16 * 4 * q < ntiles; ++q) {
    // box test: lane b takes tile 64 q + b
    const int tl = 64 * q + lane;
    bool boxfar = false, boxx = false, full = false;
    if (tl < ntiles) {
      full = jb + (tl + 1) * T <= je;  // a partial tile is never far
      const double* b = tb + 6 * (size_t)tl;
      const double gx = fmax(0.0, fmax(b[0] - rx, rx - b[3]));
      const double gy = fmax(0.0, fmax(b[1] - ry, ry - b[4]));
      const double gz = fmax(0.0, fmax(b[2] - rz, rz - b[5]));
      const double g2 = gx * gx + gy * gy + gz * gz;
      boxfar = full && g2 >= far2;
      boxx = full && g2 >= farx2;
    }
    unsigned long long fbits = __ballot(boxfar);
    const unsigned long long xbits = __ballot(boxx);
    unsigned long long todo = __ballot(full && !boxfar);
    // full tiles the box test left open, source by source, four at a time: the lanes of quarter g
    // take the g-th of them, every lane a sixteenth of its sources
    const int g = lane >> 4, r = lane & 15;
    while (todo) {
      int t[4] = {-1, -1, -1, -1};  // wave-uniform: the next (up to) four open tiles
#pragma unroll
      for (int h = 0; h < 4; ++h)
        if (todo) {
          t[h] = __ffsll(todo) - 1;
          todo &= todo - 1;
        }
      const int mine = g == 0 ? t[0] : g == 1 ? t[1] : g == 2 ? t[2] : t[3];
      bool ok = true;
      if (mine >= 0) {
        const int j0 = jb + (64 * q + mine) * T;
        for (int m = r; m < T; m += 16) {
          const double4 p = a.spos[c.off + j0 + m];
          const double ex = p.x - rx, ey = p.y - ry, ez = p.z - rz;
          ok = ok && ex * ex + ey * ey + ez * ez >= far2;
        }
      }
      const unsigned long long bad = __ballot(!ok);
#pragma unroll
      for (int h = 0; h < 4; ++h)
        if (t[h] >= 0 && ((bad >> (16 * h)) & 0xffffull) == 0) fbits |= 1ull << t[h];
    }
    // words 4 q .. 4 q + 3 (16 tiles each): bit 2b = far, bit 2b + 1 = expanded (only box-far
    // tiles are expanded)
    const int w = 4 * q + lane;
    if (lane < 4 && w < nwords) {
      a.farflags[item.flag0 + w] = spread_even((unsigned)(fbits >> (16 * lane)) & 0xffffu) |
                                   (spread_even((unsigned)(xbits >> (16 * lane)) & 0xffffu) << 1);
    }
  }
}

}  // namespace

hipError_t launch_sort(const Args& a, int B, hipStream_t s) {
  hipLaunchKernelGGL(k_keys, dim3(a.nchunks), dim3(kBlock), 0, s, a);
  int src = 0;
  for (int shift = 0; shift < 3 * kRadixBits; shift += kRadixBits) {
    hipLaunchKernelGGL(k_rhist, dim3(a.nstiles), dim3(kBlock), 0, s, a, src, shift);
    hipLaunchKernelGGL(k_rscan, dim3(B), dim3(kRadix), 0, s, a);
    hipLaunchKernelGGL(k_rscatter, dim3(a.nstiles), dim3(kBlock), 0, s, a, src, shift);
    src ^= 1;
  }
  // three passes: the sorted order is in buffer 1
  hipLaunchKernelGGL(k_gather, dim3(a.nchunks), dim3(kBlock), 0, s, a);
  const int waves = kBlock / 64;
  hipLaunchKernelGGL(k_tileboxes, dim3((a.ntboxes + waves - 1) / waves), dim3(kBlock), 0, s, a, B, a.ntboxes);
  hipLaunchKernelGGL(k_farflags, dim3((a.nitems + waves - 1) / waves), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace nb
