// Host runtime and C ABI of libnbody (include/nbody.h): argument validation (host only, before
// any HIP call), launch planning for ragged batches, workspace layout, kernel sequencing of the
// integrators, pinned staging of the per-call tables, and optional per-kernel event timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/nbody.h"
#include "nb_internal.h"

using namespace nb;

static_assert(nb::kGalaxyHernquistLog == NB_GALAXY_HERNQUIST_LOG &&
                  nb::kGalaxyAllenSantillan == NB_GALAXY_ALLEN_SANTILLAN,
              "galaxy model numbers of the kernels and of the C interface");

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(NB_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kMaxRounds = 64;  // rounds one nbody_substeps call may carry
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// The 6th-order composition of Sect. 3.1 (Yoshida 1990, solution A): drift weights of the 7
// leapfrog stages and the 8 merged kick weights.
struct Sym6 {
  double d[7], k[8];
  Sym6() {
    const double w1 = -1.17767998417887, w2 = 0.235573213359357, w3 = 0.784513610477560;
    const double w0 = 1.0 - 2.0 * (w1 + w2 + w3);
    const double w[7] = {w3, w2, w1, w0, w1, w2, w3};
    for (int i = 0; i < 7; ++i) d[i] = w[i];
    k[0] = 0.5 * w[0];
    for (int i = 1; i < 7; ++i) k[i] = 0.5 * (w[i - 1] + w[i]);
    k[7] = 0.5 * w[6];
  }
};
const Sym6 kSym6;

// Scratch of the no-allocation entry point (nbody_accel_noalloc): a fixed array in this source's
// code object, so each GPU the library runs on holds its own copy from module load until the
// process ends.  Host code must never pass `scratch` itself to a kernel or copy (on the host the
// name is a stand-in, not a device address): the address of each device's copy is looked up once
// per device with hipGetSymbolAddress and kept in g_scratch.
constexpr size_t kScratchBytes = NB_NOALLOC_SCRATCH_BYTES;
constexpr size_t kScratchTableBytes = NB_NOALLOC_TABLE_BYTES;  // pinned staging of its tables
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Workspace layout of one system (depends on the system only, not on the tile choice).
struct Layout {
  size_t cl, chunks, stiles, items, counters, coef, ref, mconst, box, partials, epart, pot, eacc, part, skey, sval,
      shist, sbase, spos, ibox, tbox, flags, total;
  size_t blob;  // bytes of the uploaded prefix [cl .. counters] (the coefficients follow it)
};

struct Plan {
  int B = 0;
  long long ntot = 0;
  int nchunks = 0;
  int nstiles = 0;  // sort tiles (NB_FP32DL only)
  int ntboxes = 0;  // j-tile box slots (NB_FP32DL only)
  int maxn = 0;
  bool anymask = false;
  bool anysplit = false;  // some cluster is finished by the combine pass (split, or kFlagDefer)
  std::vector<DevCluster> cl;
  std::vector<Chunk> chunks;
  std::vector<Chunk> stiles;
  Layout L{};
};

struct Slot {
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool used = false;
};

// j-ranges a cluster's sum is split into: enough work items for small clusters to occupy the chip
// on their own, and short enough items for the persistent grid to balance large ones (about
// 2^22 / N ranges, a power of two, at most 8 below 2^15 particles and at most 16 from there on,
// each range at least 128 sources).
// Depends on N only, so a cluster's arithmetic never depends on the batch it is in.
#ifndef NB_MIN_RANGE
#define NB_MIN_RANGE 128  // fewest sources in one j-range of a split cluster (a tuning constant)
#endif
#ifndef NB_SPLIT_CAP
#define NB_SPLIT_CAP (1LL << 22)  // bound on N x ranges (partial sums kept per cluster)
#endif
constexpr int kMaxSplit = 16;          // ranges of clusters of at least kSplit16 particles
constexpr int kSplit16 = 1 << 15;      // (smaller clusters: at most 8)
int split_of(int n) {
  const int smax = n >= kSplit16 ? kMaxSplit : 8;
  int s = 1;
  while (s < smax && (long long)n * (2 * s) <= NB_SPLIT_CAP && n / (2 * s) >= NB_MIN_RANGE) s *= 2;
  return s;
}

// far-tile words of one item's j-range: two bits per tile, 16 tiles per word
long long flag_words(int len, int T) { return ((long long)(len + T - 1) / T + 15) / 16; }

int size_class(int maxn) { return maxn < 2048 ? 0 : maxn < 32768 ? 1 : maxn < 131072 ? 2 : 3; }
int family_of(int prec) {
  return prec == NB_FP64 ? FAM_F64 : prec == NB_FP32DS ? FAM_DS : prec == NB_FP32DL ? FAM_DL : FAM_F32;
}

}  // namespace

// One captured integrator step (all stages of one leapfrog or sym6 step) and the kernel-argument
// key it was captured with; replayed nsteps times.
struct StepGraph {
  std::vector<unsigned char> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;  // recorded after its last replays; waited on before it is destroyed
};

struct nbody_ctx {
  int device = 0;
  void* scratch = nullptr;  // device address of this device's copy of `scratch`
  Slot fixed;               // pinned staging of the no-allocation entry point, allocated at creation
  int cus = 256;
  bool graphs = true;  // step graphs (nbody_use_graphs)
  hipStream_t gstream = nullptr;  // non-blocking stream the step graphs are captured on
  std::vector<StepGraph> gcache;  // small LRU cache of captured graphs (most recent last)
  TileCfg tiles[kFamilies][kSizeClasses];
  Slot slots[4];
  int next_slot = 0;
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  std::vector<hipEvent_t> event_pool;
  double ms_acc = 0.0;
  int64_t launches = 0;
  Plan plan;
  std::vector<unsigned char> blob;
};

namespace {

// RAII switch to the context's device for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}

// Host-only validation of a system description.
int check_system(const nbody_system* sys) {
  if (!sys) return fail(NB_ERR_ARG, "system is NULL");
  if (sys->nclusters < 1) return fail(NB_ERR_ARG, "nclusters must be >= 1 (got %d)", sys->nclusters);
  if (!sys->offsets) return fail(NB_ERR_ARG, "offsets is NULL");
  if (!sys->eps) return fail(NB_ERR_ARG, "eps is NULL");
  if (sys->offsets[0] != 0) return fail(NB_ERR_ARG, "offsets[0] must be 0");
  for (int b = 0; b < sys->nclusters; ++b) {
    const long long n = sys->offsets[b + 1] - sys->offsets[b];
    if (n < 1) return fail(NB_ERR_ARG, "cluster %d is empty or offsets decrease", b);
    if (n > (1LL << 30)) return fail(NB_ERR_ARG, "cluster %d has %lld particles (max 2^30)", b, n);
    const double e = sys->eps[b];
    if (!(std::isfinite(e) && e >= 0.0)) return fail(NB_ERR_ARG, "eps[%d] must be finite and >= 0", b);
  }
  if (!(std::isfinite(sys->G) && sys->G > 0.0)) return fail(NB_ERR_ARG, "G must be finite and > 0");
  if (sys->prec < NB_FP32 || sys->prec > NB_FP32DL) return fail(NB_ERR_ARG, "unknown precision mode %d", sys->prec);
  bool anyfield = false;
  if (sys->field)
    for (int b = 0; b < sys->nclusters; ++b) anyfield |= sys->field[b] != 0;
  if (anyfield) {
    const nbody_galaxy& g = sys->galaxy;
    if (g.model != NB_GALAXY_HERNQUIST_LOG && g.model != NB_GALAXY_ALLEN_SANTILLAN)
      return fail(NB_ERR_ARG, "unknown galaxy model %d", g.model);
    const bool as91 = g.model == NB_GALAXY_ALLEN_SANTILLAN;
    const double v[12] = {g.Mb, g.ab, g.Md, g.ad, g.bd, g.vh, g.dh, g.Mbh, g.ebh, g.Mh, g.ah, g.rcut};
    for (double x : v)
      if (!std::isfinite(x)) return fail(NB_ERR_ARG, "galaxy parameters must be finite");
    if (g.Mb < 0 || g.Md < 0 || g.ad < 0 || g.Mbh < 0 || g.ebh < 0)
      return fail(NB_ERR_ARG, "galaxy masses, ad and ebh must be >= 0");
    if (!(g.ab > 0 && g.bd > 0)) return fail(NB_ERR_ARG, "galaxy ab and bd must be > 0");
    if (!as91 && !(g.vh >= 0 && g.dh > 0)) return fail(NB_ERR_ARG, "galaxy vh must be >= 0 and dh > 0");
    if (as91 && !(g.Mh >= 0 && g.ah > 0 && g.rcut > 0))
      return fail(NB_ERR_ARG, "galaxy Mh must be >= 0, ah and rcut > 0");
  }
  return NB_OK;
}

Layout make_layout(int B, long long ntot, int nchunks, long long nitems_max, long long npart, int nstiles,
                   long long nflagwords, long long ntiles) {
  Layout L{};
  size_t o = 0;
  L.cl = o;
  o = align_up(o + sizeof(DevCluster) * B);
  L.chunks = o;
  o = align_up(o + sizeof(Chunk) * nchunks);
  L.stiles = o;
  o = align_up(o + sizeof(Chunk) * nstiles);
  L.items = o;
  o = align_up(o + sizeof(PairItem) * nitems_max);
  L.counters = o;  // [B] chunk counters, the item counter, the finished-blocks counter
  o = align_up(o + sizeof(int) * (B + 2));
  L.coef = o;  // [kMaxRounds][B][3] per-cluster stage coefficients; only the used rounds are uploaded
  L.blob = o;
  o = align_up(o + sizeof(double) * 3 * (size_t)B * kMaxRounds);
  L.ref = o;
  o = align_up(o + sizeof(double4) * B);
  L.mconst = o;
  o = align_up(o + sizeof(double) * B);
  L.box = o;
  o = align_up(o + sizeof(double) * 6 * B);
  L.partials = o;
  o = align_up(o + sizeof(double) * 11 * nchunks);
  L.epart = o;
  o = align_up(o + sizeof(double) * kEnergySums * nchunks);
  L.pot = o;
  o = align_up(o + sizeof(double) * ntot);
  L.eacc = o;
  o = align_up(o + sizeof(double) * 3 * ntot);
  L.part = o;
  o = align_up(o + sizeof(double4) * npart);
  L.skey = o;  // [2][ntot] (sort tiles present only)
  o = align_up(o + (nstiles ? sizeof(unsigned) * 2 * (size_t)ntot : 0));
  L.sval = o;  // [2][ntot]
  o = align_up(o + (nstiles ? sizeof(int) * 2 * (size_t)ntot : 0));
  L.shist = o;  // [nstiles][kRadix]
  o = align_up(o + sizeof(int) * (size_t)nstiles * kRadix);
  L.sbase = o;  // [B][kRadix]
  o = align_up(o + (nstiles ? sizeof(int) * (size_t)B * kRadix : 0));
  L.spos = o;  // [ntot] sorted (x, y, z, m)
  o = align_up(o + (nstiles ? sizeof(double4) * (size_t)ntot : 0));
  L.ibox = o;  // [items] centre of each work item's i-particle box, and (3/4 diagonal)^2 (NB_FP32DL)
  o = align_up(o + (nstiles ? sizeof(double4) * (size_t)nitems_max : 0));
  L.tbox = o;  // [tiles][6] bounding box of every j-tile (NB_FP32DL)
  o = align_up(o + (nstiles ? sizeof(double) * 6 * (size_t)ntiles : 0));
  L.flags = o;  // far-tile bits of every work item's j-tiles (NB_FP32DL)
  o = align_up(o + (nstiles ? sizeof(unsigned) * (size_t)nflagwords : 0));
  L.total = o;
  return L;
}

// Validate the system and build the host tables.
int build_plan(const nbody_system* sys, Plan& p) {
  int rc = check_system(sys);
  if (rc) return rc;
  p.B = sys->nclusters;
  p.cl.resize(p.B);
  p.chunks.clear();
  p.stiles.clear();
  const bool sorted = sys->prec == NB_FP32DL;
  p.maxn = 0;
  p.anymask = false;
  p.anysplit = false;
  long long nitems_max = 0, npart = 0, nflagwords = 0, ntiles = 0;
  for (int b = 0; b < p.B; ++b) {
    DevCluster& c = p.cl[b];
    c.off = sys->offsets[b];
    c.n = (int)(sys->offsets[b + 1] - sys->offsets[b]);
    const double e = sys->eps[b];
    c.eps2 = e * e;
    c.eps2f = (float)(e * e);
    c.flags = (sys->field && sys->field[b]) ? kFlagField : 0;
    // the pair kernel finishes particles in the first galaxy model only; the combine pass does both
    if ((c.flags & kFlagField) && sys->galaxy.model == NB_GALAXY_ALLEN_SANTILLAN) c.flags |= kFlagDefer;
    // FP32 rounding of a tiny eps^2 to 0 would make the self term 0 * inf; mask it then too
    const bool mask = (c.eps2 == 0.0) || (sys->prec != NB_FP64 && c.eps2f == 0.0f);
    if (mask) c.flags |= kFlagMaskSelf;
    p.anymask |= mask;
    c.chunk0 = (int)p.chunks.size();
    c.nchunks = (c.n + kChunk - 1) / kChunk;
    for (int s = 0; s < c.n; s += kChunk) p.chunks.push_back(Chunk{b, s, std::min(kChunk, c.n - s), 0});
    c.split = split_of(c.n);
    c.jlen = (c.n + c.split - 1) / c.split;
    const bool via_combine = c.split > 1 || (c.flags & kFlagDefer);
    c.part_off = via_combine ? npart : 0;
    if (via_combine) {
      npart += (long long)c.split * c.n;
      p.anysplit = true;
    }
    nitems_max += (long long)((c.n + 63) / 64) * c.split;  // the smallest item tile is 64 particles
    // far-tile words of those items: two bits per j-tile of the item's range (tiles of at least 128)
    nflagwords += (long long)((c.n + 63) / 64) * c.split * flag_words(c.jlen, 128);
    c.tbox0 = (int)ntiles;  // the cluster's j-tile boxes: room for split ranges of tiles of >= 128
    ntiles += (long long)c.split * ((c.jlen + 127) / 128);
    c.stile0 = (int)p.stiles.size();
    c.nstiles = 0;
    if (sorted)
      for (int s = 0; s < c.n; s += kSortTile) {
        p.stiles.push_back(Chunk{b, s, std::min(kSortTile, c.n - s), 0});
        ++c.nstiles;
      }
    p.maxn = std::max(p.maxn, c.n);
  }
  p.ntot = sys->offsets[p.B];
  p.nchunks = (int)p.chunks.size();
  p.nstiles = (int)p.stiles.size();
  p.ntboxes = (int)ntiles;
  p.L = make_layout(p.B, p.ntot, p.nchunks, nitems_max, npart, p.nstiles, nflagwords, ntiles);
  return NB_OK;
}

// Pair work items for i-tiles of 64 K (4 / W) particles (item_tile), longest j-ranges first (ties
// by cluster index).
void make_items(const Plan& p, const TileCfg& t, std::vector<PairItem>& items, bool flags) {
  std::vector<int> order(p.B);
  for (int b = 0; b < p.B; ++b) order[b] = b;
  // longest items first: the cost of an item is its j-range length
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return p.cl[x].jlen > p.cl[y].jlen; });
  items.clear();
  const int tile = item_tile(t);
  // j-range major: the blocks running at the same time stream the same sources through L2
  // in the local mode `flag0` is the item's first word of far-tile bits
  int words = 0;
  for (int b : order)
    for (int js = 0; js < p.cl[b].split; ++js) {
      const int len = std::min(p.cl[b].n - js * p.cl[b].jlen, p.cl[b].jlen);
      const int w = flags ? (int)flag_words(len, t.tile) : 0;
      for (int i0 = 0; i0 < p.cl[b].n; i0 += tile) {
        items.push_back(PairItem{b, i0, js, words});
        words += w;
      }
    }
}

Slot* get_slot(nbody_ctx* ctx, size_t bytes, int* rc) {
  Slot& s = ctx->slots[ctx->next_slot];
  ctx->next_slot = (ctx->next_slot + 1) % 4;
  *rc = NB_OK;
  if (s.used) {
    hipError_t e = hipEventSynchronize(s.ev);
    if (e != hipSuccess) {
      *rc = fail(NB_ERR_HIP, "staging wait: %s", hipGetErrorString(e));
      return nullptr;
    }
    s.used = false;
  }
  if (!s.ev && hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess) {
    *rc = fail(NB_ERR_HIP, "hipEventCreate failed");
    return nullptr;
  }
  if (s.cap < bytes) {
    if (s.host) (void)hipHostFree(s.host);
    s.host = nullptr;
    s.cap = 0;
    size_t cap = std::max<size_t>(bytes, 1 << 16);
    if (hipHostMalloc(&s.host, cap, hipHostMallocDefault) != hipSuccess) {
      *rc = fail(NB_ERR_NOMEM, "pinned staging allocation of %zu bytes failed", cap);
      return nullptr;
    }
    s.cap = cap;
  }
  return &s;
}

// Everything a call needs after validation: device tables uploaded, Args filled.
struct Prepared {
  Args a{};
  TileCfg tile{};
  int grid = 0;
  bool centred = false;
};

// The context's preallocated staging slot for `bytes` of tables: waits for its previous copy, never
// allocates (the no-allocation entry point's path).
Slot* fixed_slot(nbody_ctx* ctx, size_t bytes, int* rc) {
  Slot& s = ctx->fixed;
  *rc = NB_OK;
  if (!s.host || bytes > s.cap) {
    *rc = fail(NB_ERR_ARG, "tables of %zu bytes exceed the %zu-byte staging buffer", bytes, s.cap);
    return nullptr;
  }
  if (s.used) {
    hipError_t e = hipEventSynchronize(s.ev);
    if (e != hipSuccess) {
      *rc = fail(NB_ERR_HIP, "staging wait: %s", hipGetErrorString(e));
      return nullptr;
    }
    s.used = false;
  }
  return &s;
}

int prepare(nbody_ctx* ctx, const nbody_system* sys, void* ws, size_t ws_bytes, const double* coef3,
            Prepared& P, hipStream_t stream, int rounds = 1, bool fixed = false) {
  Plan& p = ctx->plan;
  const int fam = family_of(sys->prec);
  const TileCfg t = ctx->tiles[fam][size_class(p.maxn)];
  std::vector<PairItem> items;
  make_items(p, t, items, p.nstiles > 0);
  // host blob: [clusters | chunks | items | counters | coefficients of the used rounds]
  const Layout& L = p.L;
  const size_t coef_bytes = coef3 ? sizeof(double) * 3 * (size_t)p.B * rounds : 0;
  const size_t up = L.blob + coef_bytes;
  std::vector<unsigned char>& blob = ctx->blob;
  blob.assign(up, 0);
  memcpy(blob.data() + L.cl, p.cl.data(), sizeof(DevCluster) * p.B);
  memcpy(blob.data() + L.chunks, p.chunks.data(), sizeof(Chunk) * p.nchunks);
  if (p.nstiles) memcpy(blob.data() + L.stiles, p.stiles.data(), sizeof(Chunk) * p.nstiles);
  memcpy(blob.data() + L.items, items.data(), sizeof(PairItem) * items.size());
  if (coef3) memcpy(blob.data() + L.coef, coef3, coef_bytes);
  int rc = NB_OK;
  Slot* s = fixed ? fixed_slot(ctx, up, &rc) : get_slot(ctx, up, &rc);
  if (!s) return rc;
  memcpy(s->host, blob.data(), up);
  HIP_TRY(hipMemcpyAsync(ws, s->host, up, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipEventRecord(s->ev, stream));
  s->used = true;

  char* w = static_cast<char*>(ws);
  Args& a = P.a;
  a.cl = reinterpret_cast<const DevCluster*>(w + L.cl);
  a.chunks = reinterpret_cast<const Chunk*>(w + L.chunks);
  a.nchunks = p.nchunks;
  a.items = reinterpret_cast<const PairItem*>(w + L.items);
  a.nitems = (int)items.size();
  a.chunk_counter = reinterpret_cast<int*>(w + L.counters);
  a.item_counter = reinterpret_cast<int*>(w + L.counters) + p.B;

  a.partials = reinterpret_cast<double*>(w + L.partials);
  a.box = reinterpret_cast<double*>(w + L.box);
  a.stiles = reinterpret_cast<const Chunk*>(w + L.stiles);
  a.nstiles = p.nstiles;
  a.skey[0] = reinterpret_cast<unsigned*>(w + L.skey);
  a.skey[1] = a.skey[0] + p.ntot;
  a.sval[0] = reinterpret_cast<int*>(w + L.sval);
  a.sval[1] = a.sval[0] + p.ntot;
  a.shist = reinterpret_cast<int*>(w + L.shist);
  a.sbase = reinterpret_cast<int*>(w + L.sbase);
  a.perm = p.nstiles ? a.sval[1] : nullptr;
  a.spos = p.nstiles ? reinterpret_cast<double4*>(w + L.spos) : nullptr;
  a.ibox = p.nstiles ? reinterpret_cast<double4*>(w + L.ibox) : nullptr;
  a.tbox = p.nstiles ? reinterpret_cast<double*>(w + L.tbox) : nullptr;
  a.ntboxes = p.nstiles ? p.ntboxes : 0;
  a.farflags = p.nstiles ? reinterpret_cast<unsigned*>(w + L.flags) : nullptr;
  a.item_tile = item_tile(t);
  a.jtile = t.tile;
  a.mconst = reinterpret_cast<double*>(w + L.mconst);
  a.ref = reinterpret_cast<double4*>(w + L.ref);
  a.epart = reinterpret_cast<double*>(w + L.epart);
  a.pot_ws = reinterpret_cast<double*>(w + L.pot);
  a.eacc_ws = reinterpret_cast<double*>(w + L.eacc);
  a.part = reinterpret_cast<double4*>(w + L.part);
  a.coef = coef3 ? reinterpret_cast<double*>(w + L.coef) : nullptr;
  a.G = sys->G;
  a.gal = Galaxy{sys->galaxy.Mb,  sys->galaxy.ab,  sys->galaxy.Md,  sys->galaxy.ad,    sys->galaxy.bd,
                 sys->galaxy.vh,  sys->galaxy.dh,  sys->galaxy.Mbh, sys->galaxy.ebh,   sys->galaxy.model,
                 sys->galaxy.Mh,  sys->galaxy.ah,  sys->galaxy.rcut};
  a.prec = sys->prec;
  P.tile = t;
  P.grid = std::max(1, std::min(a.nitems, ctx->cus * t.bpc));
  P.centred = sys->prec == NB_FP32C || sys->prec == NB_FP32DS || sys->prec == NB_FP32DL;
  (void)ws_bytes;
  return NB_OK;
}

hipEvent_t pool_event(nbody_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int pair(nbody_ctx* ctx, const Prepared& P, bool potmode, bool kick, hipStream_t s) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->timing) {
    e0 = pool_event(ctx);
    e1 = pool_event(ctx);
    if (!e0 || !e1) return fail(NB_ERR_HIP, "event creation failed");
    HIP_TRY(hipEventRecord(e0, s));
  }
  hipError_t e = launch_pair(P.a, P.tile, P.grid, ctx->plan.anymask, potmode, kick, s);
  if (e != hipSuccess) return fail(NB_ERR_HIP, "pair kernel launch: %s", hipGetErrorString(e));
  if (ctx->timing) {
    HIP_TRY(hipEventRecord(e1, s));
    ctx->pending.emplace_back(e0, e1);
  }
  return NB_OK;
}

// One force evaluation of the current positions, optionally preceded by kick+drift and
// followed by a kick (the substep).  Kernel sequence: update (kick, drift, centre of mass, work
// counter) -> pair -> [combine of split clusters].
int evaluate(nbody_ctx* ctx, Prepared& P, bool update, bool potmode, bool kick, hipStream_t s) {
  hipError_t e;
  e = launch_update(P.a, ctx->plan.B, update, s);  // also clears the pair kernel's work counter
  if (e != hipSuccess) return fail(NB_ERR_HIP, "update kernel launch: %s", hipGetErrorString(e));
  if (P.a.nstiles) {
    e = launch_sort(P.a, ctx->plan.B, s);  // also the work items' boxes and far-tile bits
    if (e != hipSuccess) return fail(NB_ERR_HIP, "sort kernel launch: %s", hipGetErrorString(e));
  }
  int rc = pair(ctx, P, potmode, kick, s);
  if (rc || !ctx->plan.anysplit) return rc;
  e = launch_combine(P.a, potmode, kick, s);
  if (e != hipSuccess) return fail(NB_ERR_HIP, "combine kernel launch: %s", hipGetErrorString(e));
  return NB_OK;
}

int check_ptr(const void* p, const char* name) {
  if (!p) return fail(NB_ERR_ARG, "%s is NULL", name);
  if (!aligned(p, 8)) return fail(NB_ERR_ARG, "%s is not 8-byte aligned", name);
  return NB_OK;
}

int check_ws(const Plan& p, const void* ws, size_t ws_bytes) {
  if (!ws) return fail(NB_ERR_ARG, "workspace is NULL");
  if (!aligned(ws, kAlign)) return fail(NB_ERR_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < p.L.total)
    return fail(NB_ERR_ARG, "workspace too small: %zu bytes given, %zu needed", ws_bytes, p.L.total);
  return NB_OK;
}

// Common validation of the state arrays (distinct, non-overlapping, aligned).
int check_state(const Plan& p, const void* pos, const void* vel, const void* mass, const void* acc, const void* ws,
                size_t ws_bytes) {
  int rc;
  if ((rc = check_ptr(pos, "pos")) || (rc = check_ptr(mass, "mass")) || (rc = check_ptr(acc, "acc"))) return rc;
  if (vel && (rc = check_ptr(vel, "vel"))) return rc;
  if ((rc = check_ws(p, ws, ws_bytes))) return rc;
  const size_t n3 = 24 * (size_t)p.ntot, n1 = 8 * (size_t)p.ntot;
  struct R {
    const void* p;
    size_t n;
    const char* name;
    bool written;
  } r[5] = {{pos, n3, "pos", vel != nullptr},
            {vel, n3, "vel", true},
            {mass, n1, "mass", false},
            {acc, n3, "acc", true},
            {ws, p.L.total, "workspace", true}};
  for (int i = 0; i < 5; ++i)
    for (int j = i + 1; j < 5; ++j) {
      if (!r[i].p || !r[j].p) continue;
      if (!r[i].written && !r[j].written) continue;
      if (overlap(r[i].p, r[i].n, r[j].p, r[j].n))
        return fail(NB_ERR_ARG, "%s and %s overlap", r[i].name, r[j].name);
    }
  return NB_OK;
}

void default_tiles(nbody_ctx* ctx) {
  for (int f = 0; f < kFamilies; ++f)
    for (int c = 0; c < kSizeClasses; ++c)
      ctx->tiles[f][c] = c == 0 ? TileCfg{1, 4, 128, 8, 0}
                       : f == FAM_F32 ? TileCfg{2, 4, 256, 4, 0}
                                      : TileCfg{2, 4, 256, 8, 0};
}

// Key of a captured step: every kernel argument except the per-stage coefficients, plus dt (via
// the coefficients of the first stage), the launch shape and the kernel choice.
template <class F>
std::vector<unsigned char> graph_key(const Prepared& P, bool mask, int stages, F& set_stage) {
  std::vector<unsigned char> key;
  auto put = [&](const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    key.insert(key.end(), c, c + n);
  };
  for (int k = 0; k < stages; ++k) {
    Args a;
    memset(&a, 0, sizeof a);
    a = P.a;
    set_stage(k);
    a.kick_pre = P.a.kick_pre;
    a.drift = P.a.drift;
    a.kick_post = P.a.kick_post;
    a.coef = P.a.coef;
    put(&a.kick_pre, sizeof(double) * 3);
    put(&a.coef, sizeof(a.coef));
    if (k == 0) {
      put(&a.cl, offsetof(Args, kick_pre));
      put(&a.G, sizeof(double));
      put(&a.gal, sizeof(Galaxy));
      put(&a.prec, sizeof(int));
    }
  }
  put(&P.tile, sizeof P.tile);
  put(&P.grid, sizeof P.grid);
  put(&P.centred, sizeof P.centred);
  put(&mask, sizeof mask);
  put(&stages, sizeof stages);
  return key;
}

// Waits for a cached graph's last replays (on whatever stream they ran) and frees it.
void destroy_graph(StepGraph& g) {
  if (g.done) {
    (void)hipEventSynchronize(g.done);
    (void)hipEventDestroy(g.done);
  }
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g = StepGraph();
}

constexpr size_t kMaxGraphs = 8;
constexpr int kGraphSteps = 8;

// Launch `replays` replays of the graph of `stages` evaluations (captured once per argument set on
// the context's stream, and cached) on the caller's stream.
template <class F>
int replay_graph(nbody_ctx* ctx, Prepared& P, int stages, F& set_stage, int32_t replays, hipStream_t s) {
  int rc;
  if (!ctx->gstream) HIP_TRY(hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking));
  std::vector<unsigned char> key = graph_key(P, ctx->plan.anymask, stages, set_stage);
  auto& gs = ctx->gcache;
  size_t hit = gs.size();
  for (size_t i = 0; i < gs.size(); ++i)
    if (gs[i].key == key) hit = i;
  if (hit == gs.size()) {
    StepGraph g;
    HIP_TRY(hipStreamBeginCapture(ctx->gstream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < stages; ++k) {
      set_stage(k);
      if ((rc = evaluate(ctx, P, true, false, P.a.coef != nullptr || P.a.kick_post != 0.0, ctx->gstream))) {
        hipGraph_t dead = nullptr;
        (void)hipStreamEndCapture(ctx->gstream, &dead);
        if (dead) (void)hipGraphDestroy(dead);
        return rc;
      }
    }
    HIP_TRY(hipStreamEndCapture(ctx->gstream, &g.graph));
    HIP_TRY(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
    HIP_TRY(hipEventCreateWithFlags(&g.done, hipEventDisableTiming));
    g.key = std::move(key);
    if (gs.size() == kMaxGraphs) {
      destroy_graph(gs.front());
      gs.erase(gs.begin());
    }
    gs.push_back(std::move(g));
    hit = gs.size() - 1;
  } else if (hit != gs.size() - 1) {
    StepGraph g = std::move(gs[hit]);
    gs.erase(gs.begin() + hit);
    gs.push_back(std::move(g));
    hit = gs.size() - 1;
  }
  // replays go on the caller's stream itself (the context stream only records the capture), so they
  // are ordered with the caller's work without cross-stream events
  hipGraphExec_t exec = gs[hit].exec;
  for (int32_t r = 0; r < replays; ++r) HIP_TRY(hipGraphLaunch(exec, s));
  HIP_TRY(hipEventRecord(gs[hit].done, s));
  return NB_OK;
}

int run_steps(nbody_ctx* ctx, const nbody_system* sys, double* pos, double* vel, const double* mass, double* acc,
              double dt, int32_t nsteps, void* ws, size_t ws_bytes, void* stream, bool sym6) {
  if (!ctx) return fail(NB_ERR_ARG, "context is NULL");
  int rc = build_plan(sys, ctx->plan);
  if (rc) return rc;
  if ((rc = check_state(ctx->plan, pos, vel, mass, acc, ws, ws_bytes))) return rc;
  if (!vel) return fail(NB_ERR_ARG, "vel is NULL");
  if (!std::isfinite(dt)) return fail(NB_ERR_ARG, "dt must be finite");
  if (nsteps < 0) return fail(NB_ERR_ARG, "nsteps must be >= 0");
  if (nsteps == 0) return NB_OK;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(NB_ERR_HIP, "cannot select device %d", ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Prepared P;
  if ((rc = prepare(ctx, sys, ws, ws_bytes, nullptr, P, s))) return rc;
  P.a.pos = pos;
  P.a.vel = vel;
  P.a.acc = acc;
  P.a.mass = mass;
  P.a.pot = nullptr;
  const int stages = sym6 ? 7 : 1;
  auto set_stage = [&](int k) {
    P.a.kick_pre = (sym6 ? kSym6.k[k] : 0.5) * dt;
    P.a.drift = (sym6 ? kSym6.d[k] : 1.0) * dt;
    P.a.kick_post = (k == stages - 1) ? (sym6 ? kSym6.k[7] : 0.5) * dt : 0.0;
  };
  if (!ctx->graphs || ctx->timing || nsteps < 2) {
    for (int32_t step = 0; step < nsteps; ++step)
      for (int k = 0; k < stages; ++k) {
        set_stage(k);
        if ((rc = evaluate(ctx, P, true, false, k == stages - 1, s))) return rc;
      }
    return NB_OK;
  }
  // one graph holds up to kGraphSteps steps (graph launches cost more than a few kernel launches)
  const int gsteps = std::min<int>(nsteps, kGraphSteps);
  auto set_multi = [&](int k) { set_stage(k % stages); };
  if ((rc = replay_graph(ctx, P, gsteps * stages, set_multi, nsteps / gsteps, s))) return rc;
  if (nsteps % gsteps) return replay_graph(ctx, P, (nsteps % gsteps) * stages, set_multi, 1, s);
  return NB_OK;
}

}  // namespace

extern "C" {

const char* nbody_last_error(void) { return g_err.c_str(); }

int nbody_create(int device, nbody_ctx** out) {
  if (!out) return fail(NB_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (device < 0) return fail(NB_ERR_ARG, "device must be >= 0");
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count));
  if (device >= count) return fail(NB_ERR_ARG, "device %d does not exist (%d devices)", device, count);
  nbody_ctx* ctx = new (std::nothrow) nbody_ctx();
  if (!ctx) return fail(NB_ERR_NOMEM, "context allocation failed");
  ctx->device = device;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    ctx->cus = cus;
  default_tiles(ctx);
  // set-up of the no-allocation entry point: this device's scratch address (once per device, with
  // the device current) and the context's own pinned staging buffer
  {
    DeviceGuard g(device);
    int rc = NB_OK;
    if (!g.ok) rc = fail(NB_ERR_HIP, "cannot select device %d", device);
    if (!rc && device >= kMaxDevices) rc = fail(NB_ERR_UNSUPPORTED, "device %d: at most %d devices", device, kMaxDevices);
    if (!rc) {
      std::lock_guard<std::mutex> lock(g_scratch_mu);
      if (!g_scratch[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
          rc = fail(NB_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        else
          g_scratch[device] = ptr;
      }
      ctx->scratch = g_scratch[device];
    }
    if (!rc && hipHostMalloc(&ctx->fixed.host, kScratchTableBytes, hipHostMallocDefault) != hipSuccess) {
      ctx->fixed.host = nullptr;
      rc = fail(NB_ERR_NOMEM, "pinned staging allocation of %zu bytes failed", kScratchTableBytes);
    }
    if (!rc) ctx->fixed.cap = kScratchTableBytes;
    if (!rc && hipEventCreateWithFlags(&ctx->fixed.ev, hipEventDisableTiming) != hipSuccess)
      rc = fail(NB_ERR_HIP, "hipEventCreate failed");
    if (rc) {
      nbody_destroy(ctx);
      return rc;
    }
  }
  *out = ctx;
  return NB_OK;
}

void nbody_destroy(nbody_ctx* ctx) {
  if (!ctx) return;
  for (Slot* s : {&ctx->slots[0], &ctx->slots[1], &ctx->slots[2], &ctx->slots[3], &ctx->fixed}) {
    if (s->used && s->ev) (void)hipEventSynchronize(s->ev);
    if (s->ev) (void)hipEventDestroy(s->ev);
    if (s->host) (void)hipHostFree(s->host);
  }
  for (auto& pr : ctx->pending) {
    (void)hipEventSynchronize(pr.second);
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  for (StepGraph& g : ctx->gcache) destroy_graph(g);
  if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
  delete ctx;
}

size_t nbody_workspace_bytes(const nbody_ctx* ctx, const nbody_system* sys) {
  (void)ctx;
  Plan p;
  if (build_plan(sys, p)) return 0;
  return p.L.total;
}

size_t nbody_workspace_bytes_max(int64_t max_particles, int32_t max_clusters) {
  if (max_particles < 1 || max_clusters < 1 || max_clusters > max_particles) {
    fail(NB_ERR_ARG, "need 1 <= max_clusters <= max_particles");
    return 0;
  }
  const long long n = max_particles, B = max_clusters;
  // sum ceil(n_c/256) <= B + n/256; sum ceil(n_c/64) split_c <= 16 (B + n/64);
  // partial-sum rows: sum of split_c n_c over the clusters finished by the combine pass <=
  // min(16 n, B NB_SPLIT_CAP + n) (split_c n_c <= NB_SPLIT_CAP whenever split_c > 1, and an unsplit
  // cluster there, one in the second galaxy model, adds its n_c)
  const long long nchunks = B + n / kChunk;
  const long long nitems = kMaxSplit * (B + n / 64);
  const long long npart = std::min(kMaxSplit * n, B * (long long)NB_SPLIT_CAP + n);
  const long long nstiles = B + n / kSortTile;  // the sort of NB_FP32DL
  // far-tile words: sum over clusters of ceil(n_c/64) split_c ceil(jlen_c/2048)
  // <= (n/64 + B) (16 + (n + 16)/2048), since split_c <= 16 and split_c jlen_c <= n_c + split_c
  const long long nflagwords = (n / 64 + B) * (kMaxSplit + (n + kMaxSplit) / 2048 + 1);
  // j-tile boxes: sum over clusters of split_c ceil(jlen_c/128) <= n/128 + 17 B
  const long long ntiles = n / 128 + (kMaxSplit + 1) * B;
  return make_layout((int)B, n, (int)nchunks, nitems, npart, (int)nstiles, nflagwords, ntiles).total;
}

int64_t nbody_interactions(const nbody_system* sys) {
  if (check_system(sys)) return -1;
  int64_t tot = 0;
  for (int b = 0; b < sys->nclusters; ++b) {
    const int64_t n = sys->offsets[b + 1] - sys->offsets[b];
    tot += n * n;
  }
  return tot;
}

}  // extern "C"

namespace {

// nbody_accel after the plan is built: the caller's workspace, or the static scratch with the
// context's preallocated staging buffer (fixed).
int accel_call(nbody_ctx* ctx, const nbody_system* sys, const double* pos, const double* mass, double* acc,
               double* pot, void* ws, size_t ws_bytes, void* stream, bool fixed) {
  int rc;
  if ((rc = check_state(ctx->plan, pos, nullptr, mass, acc, ws, ws_bytes))) return rc;
  if (pot) {
    if ((rc = check_ptr(pot, "pot"))) return rc;
    const size_t n1 = 8 * (size_t)ctx->plan.ntot, n3 = 3 * n1;
    if (overlap(pot, n1, pos, n3) || overlap(pot, n1, acc, n3) || overlap(pot, n1, mass, n1) ||
        overlap(pot, n1, ws, ctx->plan.L.total))
      return fail(NB_ERR_ARG, "pot overlaps another buffer");
  }
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(NB_ERR_HIP, "cannot select device %d", ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Prepared P;
  if ((rc = prepare(ctx, sys, ws, ws_bytes, nullptr, P, s, 1, fixed))) return rc;
  P.a.pos = const_cast<double*>(pos);
  P.a.mass = mass;
  P.a.acc = acc;
  P.a.pot = pot;
  P.a.vel = nullptr;
  return evaluate(ctx, P, false, pot != nullptr, false, s);
}

}  // namespace

extern "C" {

int nbody_accel(nbody_ctx* ctx, const nbody_system* sys, const double* pos, const double* mass, double* acc,
                double* pot, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return fail(NB_ERR_ARG, "context is NULL");
  int rc = build_plan(sys, ctx->plan);
  if (rc) return rc;
  return accel_call(ctx, sys, pos, mass, acc, pot, ws, ws_bytes, stream, false);
}

int nbody_accel_noalloc(nbody_ctx* ctx, const nbody_system* sys, const double* pos, const double* mass, double* acc,
                        double* pot, void* stream) {
  // the limits are host-only checks of the system, made before anything else
  Plan local;
  Plan& p = ctx ? ctx->plan : local;
  int rc = build_plan(sys, p);
  if (rc) return rc;
  if (p.L.total > kScratchBytes)
    return fail(NB_ERR_ARG, "the system needs %zu bytes of workspace; the no-allocation scratch holds %zu",
                p.L.total, kScratchBytes);
  if (p.L.blob > kScratchTableBytes)
    return fail(NB_ERR_ARG, "the system's tables take %zu bytes; the no-allocation staging buffer holds %zu",
                p.L.blob, kScratchTableBytes);
  if (!ctx) return fail(NB_ERR_ARG, "context is NULL");
  if (!ctx->scratch) return fail(NB_ERR_HIP, "device scratch address unknown");
  return accel_call(ctx, sys, pos, mass, acc, pot, ctx->scratch, kScratchBytes, stream, true);
}

int nbody_substeps(nbody_ctx* ctx, const nbody_system* sys, double* pos, double* vel, const double* mass,
                   double* acc, const double* coef, int32_t nrounds, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return fail(NB_ERR_ARG, "context is NULL");
  int rc = build_plan(sys, ctx->plan);
  if (rc) return rc;
  if ((rc = check_state(ctx->plan, pos, vel, mass, acc, ws, ws_bytes))) return rc;
  if (!vel) return fail(NB_ERR_ARG, "vel is NULL");
  if (!coef) return fail(NB_ERR_ARG, "coefficient table is NULL");
  if (nrounds < 1 || nrounds > kMaxRounds) return fail(NB_ERR_ARG, "nrounds must be in [1, %d]", kMaxRounds);
  const int B = ctx->plan.B;
  for (size_t q = 0; q < 3 * (size_t)B * nrounds; ++q)
    if (!std::isfinite(coef[q]))
      return fail(NB_ERR_ARG, "coefficient %zu (round %zu, cluster %zu) is not finite", q, q / (3 * B), (q / 3) % B);
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(NB_ERR_HIP, "cannot select device %d", ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Prepared P;
  if ((rc = prepare(ctx, sys, ws, ws_bytes, coef, P, s, nrounds))) return rc;
  P.a.pos = pos;
  P.a.vel = vel;
  P.a.acc = acc;
  P.a.mass = mass;
  P.a.pot = nullptr;
  double* base = P.a.coef;
  auto set_round = [&](int r) { P.a.coef = base + 3 * (size_t)B * r; };
  if (!ctx->graphs || ctx->timing || nrounds < 2) {
    for (int r = 0; r < nrounds; ++r) {
      set_round(r);
      if ((rc = evaluate(ctx, P, true, false, true, s))) return rc;
    }
    return NB_OK;
  }
  return replay_graph(ctx, P, nrounds, set_round, 1, s);
}

int nbody_substep(nbody_ctx* ctx, const nbody_system* sys, double* pos, double* vel, const double* mass,
                  double* acc, const double* kick_pre, const double* drift, const double* kick_post, void* ws,
                  size_t ws_bytes, void* stream) {
  if (!ctx) return fail(NB_ERR_ARG, "context is NULL");
  int rc = check_system(sys);
  if (rc) return rc;
  if (!kick_pre || !drift || !kick_post) return fail(NB_ERR_ARG, "coefficient arrays must not be NULL");
  const int B = sys->nclusters;
  std::vector<double> coef(3 * (size_t)B);
  for (int b = 0; b < B; ++b) {
    coef[3 * b] = kick_pre[b];
    coef[3 * b + 1] = drift[b];
    coef[3 * b + 2] = kick_post[b];
  }
  return nbody_substeps(ctx, sys, pos, vel, mass, acc, coef.data(), 1, ws, ws_bytes, stream);
}

int nbody_step_leapfrog(nbody_ctx* ctx, const nbody_system* sys, double* pos, double* vel, const double* mass,
                        double* acc, double dt, int32_t nsteps, void* ws, size_t ws_bytes, void* stream) {
  return run_steps(ctx, sys, pos, vel, mass, acc, dt, nsteps, ws, ws_bytes, stream, false);
}

int nbody_step_sym6(nbody_ctx* ctx, const nbody_system* sys, double* pos, double* vel, const double* mass,
                    double* acc, double dt, int32_t nsteps, void* ws, size_t ws_bytes, void* stream) {
  return run_steps(ctx, sys, pos, vel, mass, acc, dt, nsteps, ws, ws_bytes, stream, true);
}

int nbody_energy(nbody_ctx* ctx, const nbody_system* sys, const double* pos, const double* vel, const double* mass,
                 double* out, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return fail(NB_ERR_ARG, "context is NULL");
  int rc = build_plan(sys, ctx->plan);
  if (rc) return rc;
  // out plays the role of the written array in the overlap checks
  if ((rc = check_ptr(out, "out"))) return rc;
  if ((rc = check_ptr(vel, "vel"))) return rc;
  if ((rc = check_state(ctx->plan, pos, nullptr, mass, vel, ws, ws_bytes))) return rc;
  const size_t no = kEnergyOut * 8 * (size_t)ctx->plan.B, n3 = 24 * (size_t)ctx->plan.ntot;
  if (overlap(out, no, pos, n3) || overlap(out, no, vel, n3) || overlap(out, no, mass, n3 / 3) ||
      overlap(out, no, ws, ctx->plan.L.total))
    return fail(NB_ERR_ARG, "out overlaps another buffer");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(NB_ERR_HIP, "cannot select device %d", ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Prepared P;
  if ((rc = prepare(ctx, sys, ws, ws_bytes, nullptr, P, s))) return rc;
  P.a.pos = const_cast<double*>(pos);
  P.a.vel = const_cast<double*>(vel);
  P.a.mass = mass;
  P.a.acc = P.a.eacc_ws;  // internal accelerations, for the force sums
  P.a.internal_only = 1;
  P.a.pot = P.a.pot_ws;
  P.a.eout = out;
  if ((rc = evaluate(ctx, P, false, true, false, s))) return rc;
  hipError_t e = launch_energy(P.a, s);
  if (e != hipSuccess) return fail(NB_ERR_HIP, "energy kernel launch: %s", hipGetErrorString(e));
  return NB_OK;
}

int nbody_set_tile(nbody_ctx* ctx, int32_t prec, int32_t nclass, nbody_tile tile) {
  if (!ctx) return fail(NB_ERR_ARG, "context is NULL");
  if (prec < NB_FP32 || prec > NB_FP32DL) return fail(NB_ERR_ARG, "unknown precision mode %d", prec);
  if (nclass < 0 || nclass >= kSizeClasses) return fail(NB_ERR_ARG, "size class must be 0, 1, 2 or 3");
  TileCfg t{tile.k, tile.waves_per_group, tile.tile, tile.blocks_per_cu, tile.phased};
  const int fam = family_of(prec);
  if (!tile_supported(fam, t))
    return fail(NB_ERR_ARG, "tile (k=%d, w=%d, tile=%d, blocks_per_cu=%d, phased=%d) is not compiled in", t.k, t.w,
                t.tile, t.bpc, t.phase);
  ctx->tiles[fam][nclass] = t;
  return NB_OK;
}

int nbody_get_tile(const nbody_ctx* ctx, int32_t prec, int32_t nclass, nbody_tile* tile) {
  if (!ctx || !tile) return fail(NB_ERR_ARG, "NULL argument");
  if (prec < NB_FP32 || prec > NB_FP32DL) return fail(NB_ERR_ARG, "unknown precision mode %d", prec);
  if (nclass < 0 || nclass >= kSizeClasses) return fail(NB_ERR_ARG, "size class must be 0, 1, 2 or 3");
  const TileCfg& t = ctx->tiles[family_of(prec)][nclass];
  tile->k = t.k;
  tile->waves_per_group = t.w;
  tile->tile = t.tile;
  tile->blocks_per_cu = t.bpc;
  tile->phased = t.phase;
  return NB_OK;
}

int nbody_sym6_coefficients(double* drift7, double* kick8) {
  if (!drift7 || !kick8) return fail(NB_ERR_ARG, "NULL argument");
  for (int i = 0; i < 7; ++i) drift7[i] = kSym6.d[i];
  for (int i = 0; i < 8; ++i) kick8[i] = kSym6.k[i];
  return NB_OK;
}

int nbody_use_graphs(nbody_ctx* ctx, int enable) {
  if (!ctx) return fail(NB_ERR_ARG, "context is NULL");
  ctx->graphs = enable != 0;
  return NB_OK;
}

int nbody_timing_enable(nbody_ctx* ctx, int enable) {
  if (!ctx) return fail(NB_ERR_ARG, "context is NULL");
  ctx->timing = enable != 0;
  return NB_OK;
}

int nbody_timing_read(nbody_ctx* ctx, double* ms_total, int64_t* launches) {
  if (!ctx || !ms_total || !launches) return fail(NB_ERR_ARG, "NULL argument");
  DeviceGuard g(ctx->device);
  for (auto& pr : ctx->pending) {
    HIP_TRY(hipEventSynchronize(pr.second));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
    ctx->ms_acc += ms;
    ctx->launches += 1;
    ctx->event_pool.push_back(pr.first);
    ctx->event_pool.push_back(pr.second);
  }
  ctx->pending.clear();
  *ms_total = ctx->ms_acc;
  *launches = ctx->launches;
  ctx->ms_acc = 0.0;
  ctx->launches = 0;
  return NB_OK;
}

}  // extern "C"
