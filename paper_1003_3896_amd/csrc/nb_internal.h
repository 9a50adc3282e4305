// Internal types shared by the gfx950 kernels and the host runtime of libnbody.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nb {

// Threads per block of every kernel, and particles per O(N) chunk (one per thread).
constexpr int kBlock = 256;
constexpr int kChunk = 256;

// Precision families of the pair kernel (FAM_DL: double-single near j-tiles, FP32 on coordinates
// centred on the i-tile for far ones, particles in Hilbert-curve order).
enum Family { FAM_F32 = 0, FAM_DS = 1, FAM_F64 = 2, FAM_DL = 3 };
constexpr int kFamilies = 4;
// Cluster-size classes of the launch-shape table (largest cluster < 2048, < 32768, < 131072, larger).
constexpr int kSizeClasses = 4;

// Hilbert-curve sort of the NB_FP32DL mode: particles per sort tile (one block), radix digit bits.
constexpr int kSortTile = 2048;
constexpr int kRadixBits = 10;
constexpr int kRadix = 1 << kRadixBits;

// Per-cluster descriptor in device memory (uploaded with every call).
struct DevCluster {
  long long off;       // first particle of the cluster in the concatenated arrays
  long long part_off;  // first row of the cluster's partial sums ([split][n] rows), when split > 1
                       // or kFlagDefer
  int n;               // particles
  int flags;           // kFlagField | kFlagMaskSelf | kFlagDefer
  double eps2;         // eps^2 in FP64
  float eps2f;         // eps^2 rounded to FP32
  int chunk0;          // first O(N) chunk of the cluster
  int nchunks;         // O(N) chunks of the cluster
  int split;           // the j-sum of every particle is split into this many ranges (1 = none)
  int jlen;            // sources per range (the last range may be shorter)
  int stile0;          // first sort tile of the cluster (NB_FP32DL)
  int nstiles;         // sort tiles of the cluster
  int tbox0;           // first j-tile box of the cluster (NB_FP32DL; room for split x ceil(jlen/128))
  int pad0;
};
constexpr int kFlagField = 1;     // add the galaxy field
constexpr int kFlagMaskSelf = 2;  // eps == 0: the j = i term must be excluded explicitly
constexpr int kFlagDefer = 4;     // finished by the combine pass even when unsplit (its galaxy model
                                  // is one the pair kernel leaves out)

// O(N) chunk: kChunk consecutive particles of one cluster (also used for sort tiles of
// kSortTile particles).
struct Chunk {
  int cluster, start, count, pad;
};

// Diagnostics: sums reduced per cluster by the energy pass, and doubles written per cluster.
constexpr int kEnergySums = 17;
constexpr int kEnergyOut = 20;

// Pair work item: one i-tile of one cluster against one j-range (js) of it.  In the local mode
// `flag0` is the item's first word of far-tile bits (bits 2t and 2t + 1 of the item's words: its
// j-tile t is far, and far enough for the expanded form of r^2).
struct PairItem {
  int cluster, i0, js, flag0;
};

// Galaxy models (the values of the C interface's NB_GALAXY_* constants).
constexpr int kGalaxyHernquistLog = 0, kGalaxyAllenSantillan = 1;
struct Galaxy {
  double Mb, ab, Md, ad, bd, vh, dh, Mbh, ebh;
  int model;  // kGalaxyHernquistLog or kGalaxyAllenSantillan
  double Mh, ah, rcut;
};

// Everything the kernels of one call need; passed by value.
struct Args {
  const DevCluster* cl;
  const Chunk* chunks;
  int nchunks;
  const PairItem* items;
  int nitems;
  int* item_counter;   // dynamic work distribution of the persistent pair kernel
  int* chunk_counter;  // [B] chunks finished per cluster (last-block reductions)
  double* partials;    // [nchunks][11] chunk sums m x, m y, m z, m, count of masses != the cluster's
                       // first; then min x, y, z and max x, y, z
  double* box;         // [B][6] bounding box of each cluster (min xyz, max xyz)
  // Hilbert-curve sort (NB_FP32DL): keys and local indices (double-buffered), per-tile digit counts and
  // offsets, and the result: perm[off + l] = local index of the particle at sorted position l
  const Chunk* stiles;
  int nstiles;
  unsigned* skey[2];
  int* sval[2];
  int* shist;          // [nstiles][kRadix] digit counts, then each tile's offsets within the digit
  int* sbase;          // [B][kRadix] first destination of each digit in its cluster
  const int* perm;     // null: particles in their own order
  double4* spos;       // [Ntot] (x, y, z, m) in sorted order (NB_FP32DL), else null
  double4* ibox;       // [items] centre of each item's i-particle box, w = (3/4 diagonal)^2 (NB_FP32DL)
  double* tbox;        // [ntboxes][6] bounding box (min xyz, max xyz) of every j-tile (NB_FP32DL)
  int ntboxes;         // box slots (NB_FP32DL)
  unsigned* farflags;  // far-tile bits of every item (NB_FP32DL; item.flag0 is its first word)
  int item_tile;       // i-particles of one work item (64 K (4/W))
  int jtile;           // j-records of one LDS tile (T)
  double* mconst;      // [B] the common mass of a cluster whose masses are all equal, else 0
  double4* ref;        // [B] reference point of each cluster (centre of mass), w = total mass
  double4* part;       // partial sums (ax, ay, az, pot) of split clusters
  double* epart;       // [nchunks * kEnergySums] energy partials
  double* pot_ws;      // [Ntot] pair potential scratch for the energy pass
  double* eacc_ws;     // [Ntot * 3] internal accelerations of the energy pass
  double* coef;        // [B*3] per-cluster (kick_pre, drift, kick_post), or null
  // state
  double* pos;
  double* vel;
  double* acc;
  double* pot;
  const double* mass;
  double* eout;  // [B * kEnergyOut] energy output
  int internal_only;  // 1: the pair pass stores the internal acceleration alone (no galaxy field)
  // uniform coefficients (used when coef == null)
  double kick_pre, drift, kick_post;
  double G;
  Galaxy gal;
  int prec;  // NB_FP32 .. NB_FP64
};

// Pair-kernel launch shape: K i-particles per lane, W waves sharing an i-group, T j-records per
// LDS tile, bpc persistent blocks per CU.
struct TileCfg {
  int k, w, tile, bpc, phase;
};

// Launchers (kernels_*.hip).  All return hipSuccess or the launch error.
hipError_t launch_update(const Args& a, int B, bool update, hipStream_t s);

hipError_t launch_pair(const Args& a, const TileCfg& t, int grid, bool mask, bool potmode, bool kick,
                       hipStream_t s);
hipError_t launch_energy(const Args& a, hipStream_t s);
hipError_t launch_combine(const Args& a, bool potmode, bool kick, hipStream_t s);
// Hilbert-curve sort: leaves the permutation in sval[1] and the sorted (x, y, z, m) in spos
hipError_t launch_sort(const Args& a, int B, hipStream_t s);


bool tile_supported(int family, const TileCfg& t);
// i-particles of one pair work item for a shape
inline int item_tile(const TileCfg& t) { return 64 * t.k * (4 / t.w); }

typedef void (*PairFn)(Args, int);
PairFn pair_kernel_f32(const TileCfg& t, bool fold, bool mask, bool pot);
PairFn pair_kernel_ds(const TileCfg& t, bool fold, bool mask, bool pot);
PairFn pair_kernel_f64(const TileCfg& t, bool fold, bool mask, bool pot);
PairFn pair_kernel_dl(const TileCfg& t, bool fold, bool mask, bool pot);

// Index in the state arrays of the particle at (sorted) local position l of cluster c.
__device__ __forceinline__ long long particle_index(const Args& a, const DevCluster& c, int l) {
  return c.off + (a.perm ? a.perm[c.off + l] : l);
}

}  // namespace nb
