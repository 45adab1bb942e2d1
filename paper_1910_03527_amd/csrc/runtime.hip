// Host runtime and C ABI of the MBE-FCI library (see include/mbefci.h).
//
// The runtime plans a batch of CASCI problems ("items"): per-item determinant
// counts, arena offsets, work lists for the segmented kernels and the sigma
// tile lists grouped by active-space size; it owns the device workspaces and
// drives the Davidson iterations either for the whole batch at once (one
// launch sequence per iteration, replayed from a captured HIP graph) or one
// CASCI at a time (the per-launch baseline).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <iterator>
#include <map>
#include <memory>
#include <stdexcept>
#include <thread>
#include <string>
#include <vector>

#include "../../include/mbefci.h"
#include "common.h"
#include "launch.h"

using namespace mbefci;

namespace {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      throw Error(MBEFCI_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));      \
  } while (0)

int64_t binom_host(int n, int k) {
  if (k < 0 || n < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  // the caller's release function when the block came from its allocator
  // (null: hipMalloc)
  void (*release)(void*, void*) = nullptr;
  void* user = nullptr;
};

struct StringTab {
  int n = 0, ne = 0, L = 0;
  int64_t N = 0;
  uint32_t* link = nullptr;   // [N][L]
  uint32_t* linkT = nullptr;  // [L][N]
  uint64_t* str = nullptr;
  int32_t* pair = nullptr;
  int32_t* pairT = nullptr;
};

// Tables of a point-group blocked CASCI shape (n, na, nb, the irreps of the
// active orbitals, the target irrep): strings sorted by (irrep, bitmask),
// links and pair tables with irrep-local string indices and class-sorted pair
// positions, and the SymInfo record (see common.h).  One device block.
struct SymTab {
  int n = 0, na = 0, nb = 0, wfn = 0, La = 0, Lb = 0;
  int64_t Na = 0, Nb = 0, ndet = 0, gsize = 0;
  void* block = nullptr;
  uint64_t* strA = nullptr;
  uint64_t* strB = nullptr;
  uint32_t* linkA = nullptr;  // [Na][La]
  uint32_t* linkB = nullptr;  // [Nb][Lb]
  uint32_t* linkBT = nullptr; // [Lb][Nb] (link-major: coalesced per-thread reads)
  int32_t* pairA = nullptr;   // [Na][npair]
  int32_t* pairB = nullptr;   // [npair][Nb]
  SymInfo* info = nullptr;    // device copy
  SymInfo host{};
};

// One kernel-shape group of a plan: items with the same active size n share
// the sigma contraction kernel (its pair dimension is a template parameter).
struct Group {
  int n = 0, tn = 64, tiles_per_wg = 16;
  std::vector<Work> tiles;
  std::vector<int> item_lo, item_hi;  // per item of the plan: its tile range (or empty)
  Work* d_tiles = nullptr;
};

// One pass of a sigma sweep: a contiguous item range whose G blocks are
// written by the contraction kernels and read back by the gather before the
// next pass reuses the same G memory.
struct Pass {
  int item_lo = 0, item_hi = 0;
  std::vector<int> tile_lo, tile_hi;  // per group
  int seg_lo = 0, seg_hi = 0;
};

struct Plan {
  std::vector<Item> items;
  std::vector<Pass> passes;
  std::vector<BucketDev> buckets;
  std::vector<Work> chunks, blocks;        // reduction chunks, 256-determinant blocks
  std::vector<Work> segs;                  // sigma gather: 4 row-aligned 64-segments per block
  std::vector<int> chunk_lo, chunk_hi, block_lo, block_hi, seg_lo, seg_hi;
  std::vector<Group> groups;
  std::vector<int> item_group;
  // point-group blocked items: their tables (null for plain items), the
  // per-class contraction work per padded class size, and the gather work
  // (256-determinant blocks) with each item's ranges
  struct SymGroup {
    int npc = 0;
    std::vector<Work> tiles;
    std::vector<int> item_lo, item_hi;
    Work* d_tiles = nullptr;
  };
  std::vector<const SymTab*> item_symtab;
  std::vector<SymGroup> sym_groups;
  std::vector<Work> sym_blocks;
  std::vector<int> sym_blk_lo, sym_blk_hi;
  Work* d_sym_blocks = nullptr;
  bool has_sym = false;
  int nitem = 0, nchunk = 0, nblock = 0, nseg = 0;
  int gather_lds = 0;  // LDS reserved per gather workgroup (an occupancy cap), gather_lds_bytes
  int64_t ntot = 0, gtot = 0, wtot = 0;
  int nsingle = 0;
  int64_t ndet_total = 0;
  // device
  Item* d_items = nullptr;
  Work* d_chunks = nullptr;
  Work* d_blocks = nullptr;
  Work* d_segs = nullptr;
  BucketDev* d_buckets = nullptr;
  double *V = nullptr, *S = nullptr, *diag = nullptr, *G = nullptr, *W = nullptr,
         *part = nullptr, *f = nullptr, *inc = nullptr, *ci = nullptr, *R = nullptr, *X = nullptr;
  // P-space (lowest-diagonal block of H): addresses, eigenvectors, eigenvalues,
  // Gram-Schmidt dot corrections; null when the P-space is off
  int32_t* pidx = nullptr;
  double *pQ = nullptr, *pT = nullptr, *pdots = nullptr;
  // the items of each P-space class (pspace_class), ascending; host copies
  // kept for the views' sub-ranges and while the uploads may be in flight
  std::vector<int32_t> pcls_h[kPspaceClasses];
  int32_t* pcls[kPspaceClasses] = {};
  // chunked selection of the P-space of CASCIs above kSelectChunk
  // determinants (host copies kept while the uploads may be in flight)
  std::vector<Work> psel_works;
  std::vector<int32_t> psel_slots;
  Work* psel_work = nullptr;
  int32_t* psel_slot = nullptr;
  uint64_t* psel_hi = nullptr;
  uint32_t* psel_lo = nullptr;
  ItemHam* hams = nullptr;
  DavState* st = nullptr;
  int32_t* tuple_pos = nullptr;
  int32_t* act = nullptr;  // [item][kMaxActive] active orbitals (MBE) or -1
  int* d_count = nullptr;
  int32_t* d_collect = nullptr;
  // MBE description (for the combine and the backward)
  bool is_mbe = false;
  // set once every array of the plan is allocated and filled: a call that
  // fails before that leaves a plan nothing may reuse
  bool ready = false;
  bool tuned = false;
  MbeSpaces sp{};
  int max_order = 0, norb = 0;
  int64_t ntuples = 0;
  std::vector<int> xsorted;
  // graph of `graph_iters` batched iterations
  hipGraphExec_t graph = nullptr;
  int graph_iters = 0;
  std::string signature;
};

}  // namespace

namespace mbefci {
hipError_t noalloc_init(int device);
int noalloc_sigma(int device, int n, int na, int nb, const double* h1, const double* eri,
                  double e_core, const double* c, double* sigma, hipStream_t s, std::string* why);
}  // namespace mbefci

struct mbefci_ctx {
  int device = 0;
  mbefci_opts opts{};
  std::string err;
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, t0 = nullptr, t1 = nullptr;
  std::map<std::pair<int, int>, StringTab> tabs;
  std::map<std::string, SymTab> symtabs;
  std::map<std::string, DevBuf> bufs;
  // workspace allocator of the caller (mbefci_set_allocator), or hipMalloc
  void* (*alloc_fn)(size_t, void*) = nullptr;
  void (*release_fn)(void*, void*) = nullptr;
  void* alloc_user = nullptr;
  std::unique_ptr<Plan> plan;
  // autotuned sigma-contraction schedule per active size n: (tile width,
  // tiles per workgroup); loaded from / saved to opts.tune_cache when set
  std::map<int, std::pair<int, int>> tuned;
  bool cache_loaded = false;
  double ms_tune = 0.0;
  bool have_forward = false;
  std::vector<double> host_scratch;
  // last screened expansion: computed tuples (masks, ascending) and their
  // increments, per order
  std::vector<std::vector<uint64_t>> scr_masks;
  std::vector<std::vector<double>> scr_inc;
};

namespace {

// Bounds of one solve batch of the screened expansion: an order with more
// tuples (or determinants) is solved in several batches.  The item bound is
// the default of opts.screen_batch.  2^16 items keep the
// per-item P-space blocks at 6.6 GB; 2^25 determinants keep the Davidson
// vectors at 9 GB and G at most 28 GB (14 active orbitals).
constexpr int64_t kScreenChunkItems = (int64_t)1 << 16;
constexpr int64_t kScreenChunkDets = (int64_t)1 << 25;

// ------------------------------------------------------------ device memory
// Free one workspace block the way it was allocated.  A block of the caller's
// allocator is handed back only after the library stream has finished every
// queued use of it (hipFree synchronises by itself).
void release_buf(mbefci_ctx* c, DevBuf& b) {
  if (b.p) {
    if (b.release) {
      (void)hipStreamSynchronize(c->stream);
      b.release(b.p, b.user);
    } else {
      (void)hipFree(b.p);
    }
  }
  b.p = nullptr;
  b.bytes = 0;
  b.release = nullptr;
  b.user = nullptr;
}

template <class T>
T* arena(mbefci_ctx* c, const std::string& name, size_t count, bool* grown = nullptr) {
  size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  DevBuf& b = c->bufs[name];
  if (b.bytes < bytes) {
    release_buf(c, b);
    size_t total = 0;
    for (auto& kv : c->bufs) total += kv.second.bytes;
    if (c->opts.max_workspace > 0 && (int64_t)(total + bytes) > c->opts.max_workspace)
      throw Error(MBEFCI_ENOMEM, "workspace cap exceeded by arena '" + name + "'");
    if (c->alloc_fn) {
      b.p = c->alloc_fn(bytes, c->alloc_user);
      if (!b.p)
        throw Error(MBEFCI_ENOMEM, "the caller's allocator returned no block of " +
                                       std::to_string(bytes) + " bytes for '" + name + "'");
      b.release = c->release_fn;
      b.user = c->alloc_user;
    } else if (hipMalloc(&b.p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      b.p = nullptr;
      throw Error(MBEFCI_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes for '" + name +
                                     "' failed");
    }
    b.bytes = bytes;
    if (grown) *grown = true;
  }
  return static_cast<T*>(b.p);
}

template <class T>
void upload(mbefci_ctx* c, T* dst, const std::vector<T>& src) {
  if (!src.empty())
    HIPCHK(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice,
                          c->stream));
}

const StringTab& string_tab(mbefci_ctx* c, int n, int ne) {
  auto key = std::make_pair(n, ne);
  auto it = c->tabs.find(key);
  if (it != c->tabs.end()) return it->second;
  StringTab t;
  t.n = n;
  t.ne = ne;
  t.N = binom_host(n, ne);
  t.L = ne * (n - ne + 1);
  if (t.N * t.L > 0) {
    HIPCHK(hipMalloc(&t.link, sizeof(uint32_t) * t.N * t.L));
    HIPCHK(hipMalloc(&t.linkT, sizeof(uint32_t) * t.N * t.L));
    launch_links(n, ne, t.N, t.link, t.linkT, nullptr, c->stream);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipMalloc(&t.str, sizeof(uint64_t) * std::max<int64_t>(t.N, 1)));
  launch_strings(n, ne, t.N, t.str, c->stream);
  const int64_t npair = (int64_t)n * (n + 1) / 2;
  HIPCHK(hipMalloc(&t.pair, sizeof(int32_t) * std::max<int64_t>(t.N * npair, 1)));
  HIPCHK(hipMalloc(&t.pairT, sizeof(int32_t) * std::max<int64_t>(t.N * npair, 1)));
  launch_pair_table(n, ne, t.N, t.pair, t.pairT, c->stream);
  HIPCHK(hipGetLastError());
  return c->tabs[key] = t;
}

// Tables of a point-group blocked CASCI shape, built on the host (integer
// work) and cached per shape on the context.  osym: irreps of the n active
// orbitals (0..7); wfn: the target irrep.
const SymTab& sym_tab(mbefci_ctx* c, int n, int na, int nb, const int* osym, int wfn) {
  std::string key = std::to_string(n) + "," + std::to_string(na) + "," + std::to_string(nb) +
                    "," + std::to_string(wfn) + ":";
  for (int t = 0; t < n; ++t) key += (char)('0' + osym[t]);
  auto it = c->symtabs.find(key);
  if (it != c->symtabs.end()) return it->second;
  SymTab T;
  T.n = n;
  T.na = na;
  T.nb = nb;
  T.wfn = wfn;
  SymInfo& Y = T.host;
  std::memset(&Y, 0, sizeof(Y));
  Y.wfn = wfn;
  const int npair = n * (n + 1) / 2;
  Y.npair = npair;
  auto irrep = [&](uint64_t m) {
    int x = 0;
    for (; m; m &= m - 1) x ^= osym[__builtin_ctzll(m)];
    return x;
  };
  auto addr = [](uint64_t m) {
    int64_t a = 0;
    int j = 1;
    for (; m; m &= m - 1, ++j) a += binom_host(__builtin_ctzll(m), j);
    return a;
  };
  // strings of one spin sorted by (irrep, bitmask); local index per address
  struct Spin {
    std::vector<uint64_t> sorted;
    std::vector<int32_t> local;  // by address
    int32_t off[kIrreps], cnt[kIrreps];
  };
  auto make_spin = [&](int ne) {
    Spin S;
    const int64_t N = binom_host(n, ne);
    std::vector<uint64_t> all(N);
    uint64_t v = ne == 0 ? 0 : (((uint64_t)1 << ne) - 1);
    for (int64_t i = 0; i < N; ++i) {
      all[i] = v;
      if (i + 1 < N) {
        const uint64_t t = v | (v - 1);
        v = (t + 1) | (((~t & (t + 1)) - 1) >> (__builtin_ctzll(v) + 1));
      }
    }
    for (int a = 0; a < kIrreps; ++a) S.cnt[a] = 0;
    for (uint64_t m : all) ++S.cnt[irrep(m)];
    int32_t o = 0;
    for (int a = 0; a < kIrreps; ++a) {
      S.off[a] = o;
      o += S.cnt[a];
    }
    S.sorted.resize(N);
    S.local.resize(N);
    int32_t fill[kIrreps] = {0};
    for (int64_t i = 0; i < N; ++i) {  // ascending bitmask within each irrep
      const int a = irrep(all[i]);
      S.sorted[S.off[a] + fill[a]] = all[i];
      S.local[i] = fill[a]++;
    }
    return S;
  };
  const Spin A = make_spin(na), B = make_spin(nb);
  T.Na = (int64_t)A.sorted.size();
  T.Nb = (int64_t)B.sorted.size();
  for (int a = 0; a < kIrreps; ++a) {
    Y.na0[a] = A.off[a];
    Y.nac[a] = A.cnt[a];
    Y.nb0[a] = B.off[a];
    Y.nbc[a] = B.cnt[a];
  }
  Y.blk[0] = 0;
  for (int a = 0; a < kIrreps; ++a)
    Y.blk[a + 1] = Y.blk[a] + (int64_t)Y.nac[a] * Y.nbc[a ^ wfn];
  T.ndet = Y.blk[kIrreps];
  // pairs class by class (ascending pair index within a class)
  std::vector<int> pos_of(npair), pa(npair), pb(npair);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b <= a; ++b) {
      pa[a * (a + 1) / 2 + b] = a;
      pb[a * (a + 1) / 2 + b] = b;
    }
  int j = 0;
  for (int cls = 0; cls < kIrreps; ++cls) {
    Y.cls0[cls] = j;
    for (int p = 0; p < npair; ++p)
      if ((osym[pa[p]] ^ osym[pb[p]]) == cls) {
        Y.pair_of[j] = p;
        Y.cls_of[j] = (int8_t)cls;
        pos_of[p] = j++;
      }
  }
  Y.cls0[kIrreps] = j;
  // G_s blocks: class s, alpha irrep a' of the irrep-G^s space
  int64_t g = 0;
  for (int cls = 0; cls < kIrreps; ++cls) {
    const int nps = Y.cls0[cls + 1] - Y.cls0[cls];
    for (int ap = 0; ap < kIrreps; ++ap) {
      Y.gofs[cls][ap] = g;
      g += (int64_t)Y.nac[ap] * nps * Y.nbc[ap ^ wfn ^ cls];
    }
  }
  Y.gsize = g;
  T.gsize = g;
  // links and pair tables of one spin, in sorted string order
  auto make_tables = [&](const Spin& S, int ne, std::vector<uint32_t>& link,
                         std::vector<int32_t>& pair, bool pair_major) {
    const int64_t N = (int64_t)S.sorted.size();
    const int L = ne * (n - ne + 1);
    link.assign(N * L, 0u);
    pair.assign(N * npair, 0);
    for (int64_t k = 0; k < N; ++k) {
      const uint64_t m = S.sorted[k];
      const int32_t self = S.local[addr(m)];
      uint32_t* e = link.data() + k * L;
      int idx = 0;
      for (int o = 0; o < n; ++o)
        if (m >> o & 1) e[idx++] = pack_link(self, pos_of[o * (o + 1) / 2 + o], 1);
      for (int q = 0; q < n; ++q) {
        if (!(m >> q & 1)) continue;
        for (int p = 0; p < n; ++p) {
          if (m >> p & 1) continue;
          const uint64_t r = (m & ~((uint64_t)1 << q)) | ((uint64_t)1 << p);
          const int lo = std::min(p, q), hi = std::max(p, q);
          const uint64_t between = (((uint64_t)1 << hi) - 1) & ~((((uint64_t)1 << lo) << 1) - 1);
          const int sg = (__builtin_popcountll(m & between) & 1) ? -1 : 1;
          e[idx++] = pack_link(S.local[addr(r)], pos_of[pair_index(p, q)], sg);
        }
      }
      for (int jj = 0; jj < npair; ++jj) {
        const int p = Y.pair_of[jj], a = pa[p], b = pb[p];
        int32_t v = 0;
        const bool ia = m >> a & 1, ib = m >> b & 1;
        if (a == b) {
          if (ia) v = pack_pair_entry(self, 1);
        } else if (ia != ib) {
          const int q = ia ? a : b, pp = ia ? b : a;
          const uint64_t r = (m & ~((uint64_t)1 << q)) | ((uint64_t)1 << pp);
          const uint64_t between = (((uint64_t)1 << a) - 1) & ~((((uint64_t)1 << b) << 1) - 1);
          const int sg = (__builtin_popcountll(m & between) & 1) ? -1 : 1;
          v = pack_pair_entry(S.local[addr(r)], sg);
        }
        if (pair_major) pair[(int64_t)jj * N + k] = v;
        else pair[k * npair + jj] = v;
      }
    }
    return L;
  };
  std::vector<uint32_t> lA, lB;
  std::vector<int32_t> pA, pB;
  T.La = make_tables(A, na, lA, pA, false);
  T.Lb = make_tables(B, nb, lB, pB, true);
  // link-major beta copy for the gather, each string's links in ascending
  // pair position (class-major): a wave's lanes then read nearby rows of G
  std::vector<uint32_t> lBT(lB.size());
  std::vector<uint32_t> row(T.Lb);
  for (int64_t k = 0; k < T.Nb; ++k) {
    std::copy(lB.begin() + k * T.Lb, lB.begin() + (k + 1) * T.Lb, row.begin());
    std::stable_sort(row.begin(), row.end(),
                     [](uint32_t x, uint32_t y) { return link_pair(x) < link_pair(y); });
    for (int l = 0; l < T.Lb; ++l) lBT[(int64_t)l * T.Nb + k] = row[l];
  }
  // one device block: strings, links, pair tables, SymInfo (256-byte aligned parts)
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t o_sa = 0, o_sb = o_sa + al(8 * T.Na), o_la = o_sb + al(8 * T.Nb),
               o_lb = o_la + al(4 * lA.size() + 4), o_pa = o_lb + al(4 * lB.size() + 4),
               o_pb = o_pa + al(4 * pA.size() + 4), o_lt = o_pb + al(4 * pB.size() + 4),
               o_in = o_lt + al(4 * lBT.size() + 4), total = o_in + al(sizeof(SymInfo));
  HIPCHK(hipMalloc(&T.block, total));
  char* base = (char*)T.block;
  T.strA = (uint64_t*)(base + o_sa);
  T.strB = (uint64_t*)(base + o_sb);
  T.linkA = (uint32_t*)(base + o_la);
  T.linkB = (uint32_t*)(base + o_lb);
  T.pairA = (int32_t*)(base + o_pa);
  T.pairB = (int32_t*)(base + o_pb);
  T.linkBT = (uint32_t*)(base + o_lt);
  T.info = (SymInfo*)(base + o_in);
  // synchronous copies: the host vectors end with this call
  HIPCHK(hipMemcpy(T.strA, A.sorted.data(), 8 * T.Na, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(T.strB, B.sorted.data(), 8 * T.Nb, hipMemcpyHostToDevice));
  if (!lA.empty()) HIPCHK(hipMemcpy(T.linkA, lA.data(), 4 * lA.size(), hipMemcpyHostToDevice));
  if (!lB.empty()) HIPCHK(hipMemcpy(T.linkB, lB.data(), 4 * lB.size(), hipMemcpyHostToDevice));
  if (!pA.empty()) HIPCHK(hipMemcpy(T.pairA, pA.data(), 4 * pA.size(), hipMemcpyHostToDevice));
  if (!pB.empty()) HIPCHK(hipMemcpy(T.pairB, pB.data(), 4 * pB.size(), hipMemcpyHostToDevice));
  if (!lBT.empty())
    HIPCHK(hipMemcpy(T.linkBT, lBT.data(), 4 * lBT.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(T.info, &Y, sizeof(SymInfo), hipMemcpyHostToDevice));
  return c->symtabs[key] = T;
}

void load_tune_cache(mbefci_ctx* c);
// Tile widths compiled for active size n: 32 and 64 columns; 128 up to 12
// orbitals except the three-wave workgroups of 8 and 9; flattened tiles of
// 32 or 64 determinants up to 9 orbitals.
bool tile_supported(int n, int tn) {
  if (tn == 32 || tn == 64) return n >= 2 && n <= 14;
  if (tn == 128) return n >= 2 && n <= 12 && n != 8 && n != 9;
  if (tn == -32 || tn == -64) return n >= 2 && n <= 9;
  return false;
}
// The schedule of active size n: a forced tile width (opts.tile; 128 becomes
// 64 where it is not compiled), else the tuned one (a schedule read from the
// cache file applies to every plan), else the default.
int tile_for(mbefci_ctx* c, int n) {
  if (c->opts.tile == 32 || c->opts.tile == 64 || c->opts.tile == 128)
    return tile_supported(n, c->opts.tile) ? c->opts.tile : 64;
  load_tune_cache(c);
  auto it = c->tuned.find(n);
  if (it != c->tuned.end()) return it->second.first;
  return n >= 10 ? 32 : 64;  // measured defaults when nothing is tuned
}
int tpw_for(mbefci_ctx* c, int n) {
  auto it = c->tuned.find(n);
  if (c->opts.tile == 0 && it != c->tuned.end()) return it->second.second;
  return 16;
}

// tune cache: one line per active size, "n tile tiles_per_wg"
void load_tune_cache(mbefci_ctx* c) {
  if (c->cache_loaded || !c->opts.tune_cache) return;
  c->cache_loaded = true;
  FILE* f = std::fopen(c->opts.tune_cache, "r");
  if (!f) return;
  int n, tn, tpw;
  char line[128];
  while (std::fgets(line, sizeof(line), f))
    if (std::sscanf(line, "%d %d %d", &n, &tn, &tpw) == 3 && tile_supported(n, tn) &&
        tpw >= 1 && tpw <= 256)
      c->tuned[n] = {tn, tpw};
  std::fclose(f);
}
void save_tune_cache(mbefci_ctx* c) {
  if (!c->opts.tune_cache) return;
  FILE* f = std::fopen(c->opts.tune_cache, "w");
  if (!f) return;
  std::fprintf(f, "# n tile tiles_per_workgroup (sigma contraction schedule, gfx950; a negative\n"
                 "# tile is that many consecutive determinants per flattened tile)\n");
  for (auto& kv : c->tuned) std::fprintf(f, "%d %d %d\n", kv.first, kv.second.first, kv.second.second);
  std::fclose(f);
}

// --------------------------------------------------------------- planning
// Sigma-contraction work units of group gi: tiles (one alpha string x tn beta
// strings) numbered column-major, tile = block * Na + Ka; a unit covers
// tiles_per_wg alpha strings of one beta block and never crosses a block.
// With flattened tiles (tn < 0) tile f holds determinants f|tn| .. f|tn|+|tn|-1
// of the item and a unit covers tiles_per_wg consecutive tiles.
void build_tiles(Plan& P, int gi) {
  Group& g = P.groups[gi];
  g.tiles.clear();
  for (int i = 0; i < P.nitem; ++i) {
    if (P.item_group[i] != gi) continue;
    const Item& I = P.items[i];
    if (g.tn < 0) {
      const int nt = (int)((I.ndet - g.tn - 1) / -g.tn);
      g.item_lo[i] = (int)g.tiles.size();
      for (int a = 0; a < nt; a += g.tiles_per_wg)
        g.tiles.push_back(Work{i, a, std::min(a + g.tiles_per_wg, nt), 0});
      g.item_hi[i] = (int)g.tiles.size();
      continue;
    }
    const int nblk = (I.Nb + g.tn - 1) / g.tn;
    g.item_lo[i] = (int)g.tiles.size();
    for (int bk = 0; bk < nblk; ++bk)
      for (int a = 0; a < I.Na; a += g.tiles_per_wg)
        g.tiles.push_back(Work{i, bk * I.Na + a, bk * I.Na + std::min(a + g.tiles_per_wg, I.Na), 0});
    g.item_hi[i] = (int)g.tiles.size();
  }
}

// Sigma passes (contiguous item ranges whose G blocks stay below
// sigma_pass_mb): sets every item's pass-relative G offset and the pass work
// ranges; returns the largest pass's G size (doubles).
int64_t build_passes(mbefci_ctx* c, Plan& P) {
  {
    const int64_t cap = c->opts.sigma_pass_mb > 0 ? (int64_t)c->opts.sigma_pass_mb << 20 : INT64_MAX;
    P.passes.clear();
    int64_t gpass = 0, gmax = 0;
    Pass cur;
    cur.tile_lo.assign(P.groups.size(), INT32_MAX);
    cur.tile_hi.assign(P.groups.size(), 0);
    cur.seg_lo = INT32_MAX;
    cur.seg_hi = 0;
    auto close = [&](int end) {
      cur.item_hi = end;
      for (size_t g = 0; g < P.groups.size(); ++g)
        if (cur.tile_lo[g] == INT32_MAX) cur.tile_lo[g] = cur.tile_hi[g] = 0;
      if (cur.seg_lo == INT32_MAX) cur.seg_lo = cur.seg_hi = 0;
      P.passes.push_back(cur);
      gmax = std::max(gmax, gpass);
      cur = Pass();
      cur.item_lo = end;
      cur.tile_lo.assign(P.groups.size(), INT32_MAX);
      cur.tile_hi.assign(P.groups.size(), 0);
      cur.seg_lo = INT32_MAX;
      cur.seg_hi = 0;
      gpass = 0;
    };
    for (int i = 0; i < P.nitem; ++i) {
      Item& I = P.items[i];
      if (I.ndet <= 1 || I.sym) continue;
      // G rows per alpha string: the off-diagonal pairs up to kFoldMax orbitals
      const int64_t gb = (int64_t)(I.n <= kFoldMax ? I.npair - I.n : I.npair) * I.Na * g_stride(I.Nb);
      if (gpass > 0 && (((gpass + 15) & ~(int64_t)15) + gb) * 8 > cap) close(i);
      gpass = (gpass + 15) & ~(int64_t)15;  // a 128-byte line
      I.goff = gpass;
      gpass += gb;
      const int g = P.item_group[i];
      cur.tile_lo[g] = std::min(cur.tile_lo[g], P.groups[g].item_lo[i]);
      cur.tile_hi[g] = std::max(cur.tile_hi[g], P.groups[g].item_hi[i]);
      cur.seg_lo = std::min(cur.seg_lo, P.seg_lo[i]);
      cur.seg_hi = std::max(cur.seg_hi, P.seg_hi[i]);
    }
    close(P.nitem);
    return gmax;
  }
}

// Work of the point-group blocked items: per item, class s and alpha irrep
// a', tiles of one alpha string x kSymTile beta strings (16 alpha strings per
// unit, never crossing a beta block) in the group of the class's padded size;
// gather blocks of 256 determinants; G blocks after the plain items' region
// (`gtot` in, grown).
void build_sym_work(Plan& P, int64_t& gtot) {
  constexpr int TPW = 16;
  P.sym_groups.clear();
  P.sym_blocks.clear();
  P.sym_blk_lo.assign(P.nitem, 0);
  P.sym_blk_hi.assign(P.nitem, 0);
  P.has_sym = false;
  std::map<int, int> grp;
  for (int i = 0; i < P.nitem; ++i) {
    Item& I = P.items[i];
    const SymTab* sy = (int)P.item_symtab.size() > i ? P.item_symtab[i] : nullptr;
    if (!sy) continue;
    P.has_sym = true;
    P.sym_blk_lo[i] = (int)P.sym_blocks.size();
    if (I.ndet <= 1) {
      P.sym_blk_hi[i] = P.sym_blk_lo[i];
      continue;
    }
    gtot = (gtot + 15) & ~(int64_t)15;
    I.goff = gtot;
    gtot += sy->gsize;
    const SymInfo& Y = sy->host;
    for (int cls = 0; cls < kIrreps; ++cls) {
      const int nps = Y.cls0[cls + 1] - Y.cls0[cls];
      if (nps == 0) continue;
      const int npc = sym_npc(nps);
      if (!grp.count(npc)) {
        grp[npc] = (int)P.sym_groups.size();
        Plan::SymGroup g;
        g.npc = npc;
        g.item_lo.assign(P.nitem, 0);
        g.item_hi.assign(P.nitem, 0);
        P.sym_groups.push_back(g);
      }
    }
    const int64_t nblk = (I.ndet + 255) / 256;
    for (int64_t k = 0; k < nblk; ++k) P.sym_blocks.push_back(Work{i, (int32_t)k, (int32_t)k + 1, 0});
    P.sym_blk_hi[i] = (int)P.sym_blocks.size();
  }
  // tiles item by item inside each group, so every item has one range per group
  for (auto& g : P.sym_groups) {
    for (int i = 0; i < P.nitem; ++i) {
      const SymTab* sy = (int)P.item_symtab.size() > i ? P.item_symtab[i] : nullptr;
      g.item_lo[i] = (int)g.tiles.size();
      if (sy && P.items[i].ndet > 1) {
        const SymInfo& Y = sy->host;
        for (int cls = 0; cls < kIrreps; ++cls) {
          const int nps = Y.cls0[cls + 1] - Y.cls0[cls];
          if (nps == 0 || sym_npc(nps) != g.npc) continue;
          for (int ap = 0; ap < kIrreps; ++ap) {
            const int NA = Y.nac[ap], NB = Y.nbc[ap ^ Y.wfn ^ cls];
            if (NA == 0 || NB == 0) continue;
            const int TN = sym_tile(g.npc);
            const int nbk = (NB + TN - 1) / TN;
            for (int bk = 0; bk < nbk; ++bk)
              for (int a = 0; a < NA; a += TPW)
                g.tiles.push_back(Work{i, bk * NA + a, bk * NA + std::min(a + TPW, NA),
                                       cls * 8 + ap});
          }
        }
      }
      g.item_hi[i] = (int)g.tiles.size();
    }
  }
}

// items must have n, na, nb filled; computes every derived field, work lists
// and allocates the arenas.
// The P-space machinery gives every solve its guess (and solves every CASCI
// of at most kMaxPspace determinants exactly) under both corrections; its
// correction on the P block is used with the diagonal correction only.

void finalize_plan(mbefci_ctx* c, Plan& P, int nguess_slots) {
  const int mmax = c->opts.max_space;
  P.nitem = (int)P.items.size();
  int64_t off = 0, goff = 0, woff = 0;
  int chunk = 0;
  std::map<int, int> group_of_n;
  P.item_group.assign(P.nitem, -1);
  P.chunks.clear();
  P.blocks.clear();
  P.chunk_lo.assign(P.nitem, 0);
  P.chunk_hi.assign(P.nitem, 0);
  P.block_lo.assign(P.nitem, 0);
  P.block_hi.assign(P.nitem, 0);
  P.segs.clear();
  P.seg_lo.assign(P.nitem, 0);
  P.seg_hi.assign(P.nitem, 0);
  P.nsingle = 0;
  P.ndet_total = 0;
  // string tables by (n, electrons): a plan's items share few shapes
  const StringTab* tab_of[kMaxActive + 1][kMaxActive + 1] = {};
  auto tab = [&](int n, int ne) -> const StringTab& {
    const StringTab*& t = tab_of[n][ne];
    if (!t) t = &string_tab(c, n, ne);
    return *t;
  };
  for (int i = 0; i < P.nitem; ++i) {
    Item& I = P.items[i];
    if (I.n > 14) throw Error(MBEFCI_EUNSUPPORTED, "active space of " + std::to_string(I.n) +
                                                       " orbitals exceeds the compiled kernels (14)");
    const SymTab* sy = (int)P.item_symtab.size() > i ? P.item_symtab[i] : nullptr;
    if (sy) {
      I.Na = (int32_t)sy->Na;
      I.Nb = (int32_t)sy->Nb;
      I.La = sy->La;
      I.Lb = sy->Lb;
      I.linkA = sy->linkA;
      I.linkB = sy->linkB;
      I.linkBT = sy->linkBT;
      I.strA = sy->strA;
      I.strB = sy->strB;
      I.pairA = sy->pairA;
      I.pairB = sy->pairB;
      I.sym = sy->info;
      I.ndet = sy->ndet;
      if (I.ndet < 1)
        throw Error(MBEFCI_EINVAL, "no determinant of the requested irrep in a CASCI space");
    } else {
      const StringTab& ta = tab(I.n, I.na);
      const StringTab& tb = tab(I.n, I.nb);
      I.Na = (int32_t)ta.N;
      I.Nb = (int32_t)tb.N;
      I.La = ta.L;
      I.Lb = tb.L;
      I.linkA = ta.link;
      I.linkB = tb.link;
      I.linkBT = tb.linkT;
      I.strA = ta.str;
      I.strB = tb.str;
      I.pairA = ta.pair;
      I.pairB = tb.pairT;
      I.sym = nullptr;
      I.ndet = (int64_t)I.Na * I.Nb;
    }
    I.npair = I.n * (I.n + 1) / 2;
    I.kpad = (I.npair + 15) / 16 * 16;
    I.off = off;
    off += (I.ndet + 63) / 64 * 64;
    I.ham = i;
    P.ndet_total += I.ndet;
    if (I.ndet > 1) {
      goff = (goff + 15) & ~(int64_t)15;  // a 128-byte line
      I.goff = goff;
      goff += sy ? sy->gsize : (int64_t)I.npair * I.Na * g_stride(I.Nb);
      I.woff = woff;
      woff += (int64_t)I.kpad * I.kpad;
    } else {
      I.goff = 0;
      I.woff = 0;
      ++P.nsingle;
    }
    const int nch = (int)((I.ndet + kChunkElems - 1) / kChunkElems);
    I.chunk0 = chunk;
    I.nchunk = nch;
    P.chunk_lo[i] = (int)P.chunks.size();
    for (int k = 0; k < nch; ++k) P.chunks.push_back(Work{i, chunk + k, chunk + k + 1, 0});
    P.chunk_hi[i] = (int)P.chunks.size();
    chunk += nch;
    const int nbk = (int)((I.ndet + 255) / 256);
    P.block_lo[i] = (int)P.blocks.size();
    for (int k = 0; k < nbk; ++k) P.blocks.push_back(Work{i, k, k + 1, 0});
    P.block_hi[i] = (int)P.blocks.size();
    P.seg_lo[i] = (int)P.segs.size();
    if (I.ndet > 1 && !sy) {
      const int nsg = I.Na * ((I.Nb + 63) / 64);
      for (int b = 0; b * 4 < nsg; ++b) P.segs.push_back(Work{i, b, nsg, 0});
    }
    P.seg_hi[i] = (int)P.segs.size();
    if (I.ndet > 1 && !sy) {
      if (!group_of_n.count(I.n)) {
        group_of_n[I.n] = (int)P.groups.size();
        Group g;
        g.n = I.n;
        g.tn = tile_for(c, I.n);
        g.tiles_per_wg = tpw_for(c, I.n);
        g.item_lo.assign(P.nitem, 0);
        g.item_hi.assign(P.nitem, 0);
        P.groups.push_back(g);
      }
      P.item_group[i] = group_of_n[I.n];
    }
  }
  for (size_t gi = 0; gi < P.groups.size(); ++gi) build_tiles(P, (int)gi);
  goff = build_passes(c, P);
  build_sym_work(P, goff);
  P.ntot = std::max<int64_t>(off, 64);
  P.gtot = goff;
  P.wtot = woff;
  P.nchunk = (int)P.chunks.size();
  P.nblock = (int)P.blocks.size();
  P.nseg = (int)P.segs.size();
  {
    // the gather's occupancy follows the row block (npair x row stride) of
    // the items that hold most of its segments
    std::map<int64_t, int64_t> segs_by_block;
    for (int i = 0; i < P.nitem; ++i) {
      const Item& I = P.items[i];
      if (P.seg_hi[i] > P.seg_lo[i])
        segs_by_block[(int64_t)I.npair * g_stride(I.Nb) * 8] += P.seg_hi[i] - P.seg_lo[i];
    }
    int64_t best = 0, most = -1;
    for (const auto& kv : segs_by_block)
      if (kv.second > most) best = kv.first, most = kv.second;
    P.gather_lds = gather_lds_bytes(best);
  }

  bool grown = false;
  P.d_items = arena<Item>(c, "items", P.nitem, &grown);
  P.d_chunks = arena<Work>(c, "chunks", P.nchunk, &grown);
  P.d_blocks = arena<Work>(c, "blocks", P.nblock, &grown);
  P.d_segs = arena<Work>(c, "segs", P.nseg, &grown);
  P.hams = arena<ItemHam>(c, "hams", P.nitem, &grown);
  P.st = arena<DavState>(c, "state", P.nitem, &grown);
  P.V = arena<double>(c, "V", (size_t)(mmax + 1) * P.ntot, &grown);
  P.S = arena<double>(c, "S", (size_t)mmax * P.ntot, &grown);
  P.diag = arena<double>(c, "diag", P.ntot, &grown);
  {
    P.pidx = arena<int32_t>(c, "pidx", (size_t)P.nitem * kMaxPspace, &grown);
    P.pQ = arena<double>(c, "pQ", (size_t)P.nitem * kMaxPspace * kMaxPspace, &grown);
    P.pT = arena<double>(c, "pT", (size_t)P.nitem * 2 * kMaxPspace, &grown);
    P.pdots = arena<double>(c, "pdots", (size_t)P.nitem * (kMaxSpace + 1), &grown);
    for (int q = 0; q < kPspaceClasses; ++q) P.pcls_h[q].clear();
    for (int i = 0; i < P.nitem; ++i) {
      const int q = pspace_class(P.items[i].ndet, c->opts.pspace);
      if (q >= 0) P.pcls_h[q].push_back(i);
    }
    for (int q = 0; q < kPspaceClasses; ++q) {
      P.pcls[q] = arena<int32_t>(c, "pclass" + std::to_string(q),
                                 std::max<size_t>(P.pcls_h[q].size(), 1), &grown);
      upload(c, P.pcls[q], P.pcls_h[q]);
    }
    P.psel_works.clear();
    P.psel_slots.assign(P.nitem, -1);
    int32_t nslot = 0;
    for (int i = 0; i < P.nitem; ++i) {
      const int64_t nd = P.items[i].ndet;
      if (nd <= kSelectChunk) continue;
      const int nch = (int)((nd + kSelectChunk - 1) / kSelectChunk);
      P.psel_slots[i] = nslot;
      for (int k = 0; k < nch; ++k) P.psel_works.push_back(Work{i, k, nslot, 0});
      nslot += nch;
    }
    P.psel_slot = arena<int32_t>(c, "psel_slot", P.nitem, &grown);
    P.psel_work = arena<Work>(c, "psel_work", std::max<size_t>(P.psel_works.size(), 1), &grown);
    P.psel_hi = arena<uint64_t>(c, "psel_hi", (size_t)std::max(nslot, 1) * kMaxPspace, &grown);
    P.psel_lo = arena<uint32_t>(c, "psel_lo", (size_t)std::max(nslot, 1) * kMaxPspace, &grown);
    upload(c, P.psel_slot, P.psel_slots);
    upload(c, P.psel_work, P.psel_works);
  }
  // residual and Ritz vectors of the Olsen correction (every solve may switch
  // to it near convergence)
  P.R = arena<double>(c, "resid", P.ntot, &grown);
  P.X = arena<double>(c, "ritz", P.ntot, &grown);
  P.G = arena<double>(c, "G", std::max<int64_t>(P.gtot, 1), &grown);
  P.W = arena<double>(c, "W", std::max<int64_t>(P.wtot, 1), &grown);
  P.part = arena<double>(c, "part", (size_t)std::max(P.nchunk, 1) * kPartStride, &grown);
  P.f = arena<double>(c, "f", P.nitem + 2, &grown);
  P.inc = arena<double>(c, "inc", P.nitem, &grown);
  P.d_count = arena<int>(c, "count", 4, &grown);
  P.d_collect = arena<int32_t>(c, "collect", (size_t)4 * P.nitem, &grown);
  if (c->opts.keep_ci) P.ci = arena<double>(c, "ci", P.ntot, &grown);
  for (size_t g = 0; g < P.groups.size(); ++g)
    P.groups[g].d_tiles =
        arena<Work>(c, "tiles" + std::to_string(g), P.groups[g].tiles.size(), &grown);
  for (size_t g = 0; g < P.sym_groups.size(); ++g) {
    P.sym_groups[g].d_tiles = arena<Work>(c, "symtiles" + std::to_string(g),
                                          std::max<size_t>(P.sym_groups[g].tiles.size(), 1), &grown);
    upload(c, P.sym_groups[g].d_tiles, P.sym_groups[g].tiles);
  }
  if (P.has_sym) {
    P.d_sym_blocks = arena<Work>(c, "symblocks", std::max<size_t>(P.sym_blocks.size(), 1), &grown);
    upload(c, P.d_sym_blocks, P.sym_blocks);
  }
  upload(c, P.d_items, P.items);
  upload(c, P.d_chunks, P.chunks);
  upload(c, P.d_blocks, P.blocks);
  upload(c, P.d_segs, P.segs);
  for (auto& g : P.groups) upload(c, g.d_tiles, g.tiles);
  (void)nguess_slots;
}

// ----------------------------------------------------------------- solver
struct View {
  int ibase, nitem;
  int chunk_lo, nchunk;
  int seg_lo, nseg;
  int item;  // -1: whole plan, else the single item
};

View whole(const Plan& P) { return View{0, P.nitem, 0, P.nchunk, 0, P.nseg, -1}; }
View single(const Plan& P, int i) {
  return View{i, 1, P.chunk_lo[i], P.chunk_hi[i] - P.chunk_lo[i], P.seg_lo[i],
              P.seg_hi[i] - P.seg_lo[i], i};
}

// One launch of the sigma sweep: kind 0 = contraction of group `group`,
// kind 1 = gather, kind 2 = blocked contraction of sym group `group`, kind 3 =
// blocked gather; work-list range [lo, lo + cnt).
struct SigmaLaunch {
  int kind, group, lo, cnt;
};

void sym_launches(const Plan& P, int item, std::vector<SigmaLaunch>& out) {
  for (size_t g = 0; g < P.sym_groups.size(); ++g) {
    const auto& sg = P.sym_groups[g];
    const int lo = item >= 0 ? sg.item_lo[item] : 0;
    const int hi = item >= 0 ? sg.item_hi[item] : (int)sg.tiles.size();
    if (hi > lo) out.push_back({2, (int)g, lo, hi - lo});
  }
  const int lo = item >= 0 ? P.sym_blk_lo[item] : 0;
  const int hi = item >= 0 ? P.sym_blk_hi[item] : (int)P.sym_blocks.size();
  if (hi > lo) out.push_back({3, -1, lo, hi - lo});
}

std::vector<SigmaLaunch> sigma_launches(const Plan& P, const View& v) {
  std::vector<SigmaLaunch> out;
  if (v.item >= 0) {
    if (P.items[v.item].sym) {
      sym_launches(P, v.item, out);
      return out;
    }
    const int g = P.item_group[v.item];
    if (g < 0) return out;
    out.push_back({0, g, P.groups[g].item_lo[v.item],
                   P.groups[g].item_hi[v.item] - P.groups[g].item_lo[v.item]});
    out.push_back({1, -1, v.seg_lo, v.nseg});
    return out;
  }
  if (P.has_sym) sym_launches(P, -1, out);
  for (const Pass& ps : P.passes) {
    bool any = false;
    for (size_t g = 0; g < P.groups.size(); ++g)
      if (ps.tile_hi[g] > ps.tile_lo[g]) {
        out.push_back({0, (int)g, ps.tile_lo[g], ps.tile_hi[g] - ps.tile_lo[g]});
        any = true;
      }
    if (any) out.push_back({1, -1, ps.seg_lo, ps.seg_hi - ps.seg_lo});
  }
  return out;
}

void sigma_launch(mbefci_ctx* c, Plan& P, const SigmaLaunch& L, int slot) {
  if (L.kind == 0) {
    const Group& g = P.groups[L.group];
    if (!launch_sigma_dgemm(g.n, g.tn, P.d_items, g.d_tiles + L.lo, L.cnt, P.W, P.V, P.ntot, P.G,
                            P.S, P.st, slot, c->stream))
      throw Error(MBEFCI_EUNSUPPORTED, "no sigma kernel for n=" + std::to_string(g.n));
  } else if (L.kind == 1) {
    launch_sigma_gather(P.d_items, P.d_segs + L.lo, L.cnt, P.G, P.S, P.ntot, P.st, slot,
                        P.gather_lds, c->stream);
  } else if (L.kind == 2) {
    const auto& sg = P.sym_groups[L.group];
    if (!launch_sigma_sym_dgemm(sg.npc, P.d_items, sg.d_tiles + L.lo, L.cnt, P.W, P.V, P.ntot,
                                P.G, P.st, slot, c->stream))
      throw Error(MBEFCI_EUNSUPPORTED, "no blocked sigma kernel for " + std::to_string(sg.npc) +
                                           " pairs in a class");
  } else {
    launch_sigma_sym_gather(P.d_items, P.d_sym_blocks + L.lo, L.cnt, P.G, P.S, P.ntot, P.st, slot,
                            c->stream);
  }
}

void sigma(mbefci_ctx* c, Plan& P, const View& v, int slot) {
  for (const SigmaLaunch& L : sigma_launches(P, v)) sigma_launch(c, P, L, slot);
}

void add_vector(mbefci_ctx* c, Plan& P, const View& v, int slot) {
  sigma(c, P, v, slot);
  launch_dav_dots(P.d_items, P.d_chunks + v.chunk_lo, v.nchunk, P.V, P.S, P.ntot, P.st, slot,
                  P.part, c->stream);
  launch_dav_rr(P.d_items, v.ibase, v.nitem, P.part, P.st, slot, c->stream);
}

// One Davidson iteration is split in two halves so that the convergence test
// sits between them: step_a forms the residual of the current Ritz vector,
// decides convergence and builds the next basis vector; step_b applies sigma
// to it and updates the subspace matrix and Ritz pair.
constexpr double kOlsenSwitch = 1e-7;
void step_a(mbefci_ctx* c, Plan& P, const View& v) {
  const bool olsen = c->opts.precond == 1;
  const PspaceArgs ps{P.pidx, P.pQ, P.pT, P.pdots};
  // with the diagonal / P-space correction a CASCI switches to the Olsen
  // correction once its residual is below kOlsenSwitch: that correction is
  // exact on the P block, so near convergence most of the new direction lies
  // along the Ritz vector and cancels in the Gram-Schmidt step
  const double below = (!olsen && c->opts.conv_tol < kOlsenSwitch) ? kOlsenSwitch : 0.0;
  launch_dav_iteration(P.d_items, v.ibase, v.nitem, P.d_chunks + v.chunk_lo, v.nchunk, P.V, P.S,
                       P.diag, P.ntot, P.st, P.part, c->opts.conv_tol, c->opts.max_iter,
                       c->opts.max_space, P.R, P.X, (P.pidx && !olsen) ? &ps : nullptr, olsen,
                       below, c->stream);
}
void step_b(mbefci_ctx* c, Plan& P, const View& v) { add_vector(c, P, v, -1); }

int count_active(mbefci_ctx* c, Plan& P, const View& v) {
  launch_count_active(P.st, v.ibase, v.nitem, P.d_count, c->stream);
  int h = 0;
  HIPCHK(hipMemcpyAsync(&h, P.d_count, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return h;
}

// Autotuner: for every active size n of the plan that has no tuned schedule
// yet, time the contraction kernel over the group's whole work list for each
// candidate (tile width, tiles per workgroup) on the live plan (guess vectors
// in slot 0; the kernels' cost does not depend on the values) and keep the
// fastest.  Results persist in the context and, with opts.tune_cache, in a
// file.  Runs once per plan, before the iteration graph is captured.
void autotune(mbefci_ctx* c, Plan& P) {
  if (c->opts.tile != 0 || P.tuned) return;
  P.tuned = true;
  load_tune_cache(c);
  HIPCHK(hipStreamSynchronize(c->stream));  // the clock covers the tuner only
  auto t0 = std::chrono::steady_clock::now();
  bool changed = false;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  for (size_t gi = 0; gi < P.groups.size(); ++gi) {
    Group& g = P.groups[gi];
    if (c->tuned.count(g.n)) {
      if (g.tn != c->tuned[g.n].first || g.tiles_per_wg != c->tuned[g.n].second) {
        g.tn = c->tuned[g.n].first;
        g.tiles_per_wg = c->tuned[g.n].second;
        changed = true;
      }
      continue;
    }
    float best = 1e30f;
    std::pair<int, int> pick{g.tn, g.tiles_per_wg};
    for (int tn : {32, 64, 128, -32, -64}) {
      if (!tile_supported(g.n, tn)) continue;
      for (int tpw : {4, 8, 16, 32}) {
        g.tn = tn;
        g.tiles_per_wg = tpw;
        build_tiles(P, (int)gi);
        Work* d = arena<Work>(c, "tune_tiles", g.tiles.size());
        upload(c, d, g.tiles);
        const int nw = (int)g.tiles.size();
        launch_sigma_dgemm(g.n, tn, P.d_items, d, nw, P.W, P.V, P.ntot, P.G, P.S, P.st, 0,
                           c->stream);
        HIPCHK(hipEventRecord(e0, c->stream));
        for (int r = 0; r < 3; ++r)
          launch_sigma_dgemm(g.n, tn, P.d_items, d, nw, P.W, P.V, P.ntot, P.G, P.S, P.st, 0,
                           c->stream);
        HIPCHK(hipEventRecord(e1, c->stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        // a later candidate replaces the pick only when it is at least 3%
        // faster, so near-ties keep the same schedule from run to run
        if (ms < 0.97f * best) {
          best = ms;
          pick = {tn, tpw};
        }
      }
    }
    c->tuned[g.n] = pick;
    g.tn = pick.first;
    g.tiles_per_wg = pick.second;
    changed = true;
  }
  HIPCHK(hipEventDestroy(e0));
  HIPCHK(hipEventDestroy(e1));
  if (changed) {
    for (size_t gi = 0; gi < P.groups.size(); ++gi) {
      build_tiles(P, (int)gi);
      P.groups[gi].d_tiles =
          arena<Work>(c, "tiles" + std::to_string(gi), P.groups[gi].tiles.size());
      upload(c, P.groups[gi].d_tiles, P.groups[gi].tiles);
    }
    build_passes(c, P);  // item G offsets are unchanged; pass work ranges follow the tiles
    save_tune_cache(c);
  }
  c->ms_tune += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                    .count();
}

// guess + iterations for the items of view v (hdiag and set-up already done)
void solve_view(mbefci_ctx* c, Plan& P, const View& v, int* graph_launches) {
  int g = std::max(1, std::min(c->opts.nguess, 8));
  if (P.pidx) {
    const PspaceSelect sel{P.psel_work, (int)P.psel_works.size(), P.psel_slot, P.psel_hi,
                           P.psel_lo};
    PspaceLists pl{};
    for (int q = 0; q < kPspaceClasses; ++q) {
      const auto& h = P.pcls_h[q];
      const auto lo = std::lower_bound(h.begin(), h.end(), v.ibase);
      const auto hi = std::lower_bound(lo, h.end(), v.ibase + v.nitem);
      pl.list[q] = P.pcls[q] + (lo - h.begin());
      pl.n[q] = (int)(hi - lo);
    }
    launch_pspace_setup(P.d_items, v.ibase, v.nitem, pl, P.hams, P.diag, P.pidx, P.pQ, P.pT, P.V,
                        P.ntot, P.st, c->opts.pspace, g, sel, c->stream);
    g += 1;  // unit vectors (or the P-space eigenvector) and the dense vector
  } else {
    launch_dav_guess(P.d_items, v.ibase, v.nitem, P.diag, P.V, P.ntot, P.st, g, c->stream);
    g += 1;  // the dense vector
  }
  if (v.item < 0) autotune(c, P);
  for (int j = 0; j < g; ++j) add_vector(c, P, v, j);
  const int max_iter = c->opts.max_iter;
  step_a(c, P, v);
  if (v.item < 0 && c->opts.use_graph) {
    const int K = 4;
    if (count_active(c, P, v) == 0) return;
    if (!P.graph || P.graph_iters != K) {
      if (P.graph) {
        HIPCHK(hipGraphExecDestroy(P.graph));
        P.graph = nullptr;
      }
      hipGraph_t gr;
      HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < K; ++k) {
        step_b(c, P, v);
        step_a(c, P, v);
      }
      HIPCHK(hipStreamEndCapture(c->stream, &gr));
      HIPCHK(hipGraphInstantiate(&P.graph, gr, nullptr, nullptr, 0));
      HIPCHK(hipGraphDestroy(gr));
      P.graph_iters = K;
    }
    for (int it = 0; it < max_iter + K; it += K) {
      HIPCHK(hipGraphLaunch(P.graph, c->stream));
      if (graph_launches) ++*graph_launches;
      if (count_active(c, P, v) == 0) break;
    }
  } else if (v.item < 0) {
    const int K = 4;
    if (count_active(c, P, v) == 0) return;
    for (int it = 0; it < max_iter + K; it += K) {
      for (int k = 0; k < K; ++k) {
        step_b(c, P, v);
        step_a(c, P, v);
      }
      if (count_active(c, P, v) == 0) break;
    }
  } else {
    for (int it = 0; it < max_iter + 1; ++it) {
      if (count_active(c, P, v) == 0) break;
      step_b(c, P, v);
      step_a(c, P, v);
    }
  }
  HIPCHK(hipGetLastError());
}

void solve_plan(mbefci_ctx* c, Plan& P, mbefci_stats* stats) {
  const int g = std::max(1, std::min(c->opts.nguess, 8)) + 1;
  HIPCHK(hipEventRecord(c->t0, c->stream));
  launch_hdiag(P.d_items, P.d_blocks, P.nblock, P.hams, P.diag, c->stream);
  launch_fill(P.V, (int64_t)g * P.ntot, 0.0, c->stream);
  int graph_launches = 0;
  if (c->opts.mode == MBEFCI_PER_LAUNCH) {
    for (int i = 0; i < P.nitem; ++i) solve_view(c, P, single(P, i), nullptr);
  } else {
    solve_view(c, P, whole(P), &graph_launches);
  }
  if (c->opts.keep_ci)
    launch_ritz_vector(P.d_items, P.d_chunks, P.nchunk, P.V, P.ntot, P.st, P.ci, c->stream);
  HIPCHK(hipEventRecord(c->t1, c->stream));
  // statistics and convergence check
  launch_collect(P.st, P.nitem, P.d_collect, c->stream);
  std::vector<int32_t> col(4 * (size_t)P.nitem);
  HIPCHK(hipMemcpyAsync(col.data(), P.d_collect, col.size() * sizeof(int32_t),
                        hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  int first_failed = -1, max_iters = 0;
  int64_t sig = 0;
  for (int i = 0; i < P.nitem; ++i) {
    max_iters = std::max(max_iters, col[4 * i]);
    if (P.items[i].ndet > 1) sig += col[4 * i] + col[4 * i + 2];
    if (col[4 * i + 1] == 1 && first_failed < 0) first_failed = i;
  }
  if (stats) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->t0, c->t1));
    stats->ntuples = P.nitem;
    stats->nsingle = P.nsingle;
    stats->sigma_calls = sig;
    stats->ndet_total = P.ndet_total;
    stats->max_iters = max_iters;
    stats->first_failed = first_failed;
    stats->nbuckets = (int32_t)P.buckets.size();
    stats->graph_launches = graph_launches;
    stats->ms_solve = ms;
    stats->ms_tune = c->ms_tune;
  }
  if (first_failed >= 0)
    throw Error(MBEFCI_ENOTCONV, "Davidson did not converge for CASCI " +
                                     std::to_string(first_failed) + " within " +
                                     std::to_string(c->opts.max_iter) + " iterations");
}

// ------------------------------------------------------------ validation
// Validate the MO integrals on the device (finite, h symmetric, (pq|rs)
// 8-fold symmetric to 1e-12 relative); the flags word is read back before
// anything is solved.
void check_integrals(mbefci_ctx* c, int M, const double* h1, const double* eri) {
  if (!c->opts.validate) return;
  int* d_flags = arena<int>(c, "check_flags", 1);
  HIPCHK(hipMemsetAsync(d_flags, 0, sizeof(int), c->stream));
  launch_check_integrals(h1, eri, M, d_flags, c->stream);
  HIPCHK(hipGetLastError());
  int flags = 0;
  HIPCHK(hipMemcpyAsync(&flags, d_flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (flags & 1) throw Error(MBEFCI_EINVAL, "h1 holds a non-finite value");
  if (flags & 4) throw Error(MBEFCI_EINVAL, "eri holds a non-finite value");
  if (flags & 2) throw Error(MBEFCI_EINVAL, "h1 is not symmetric");
  if (flags & 8) throw Error(MBEFCI_EINVAL, "eri lacks the 8-fold permutational symmetry");
}

struct StreamScope {  // order the library stream after the caller's and back
  mbefci_ctx* c;
  hipStream_t user;
  StreamScope(mbefci_ctx* cc, void* s) : c(cc), user((hipStream_t)s) {
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipEventRecord(c->ev_in, user));
    HIPCHK(hipStreamWaitEvent(c->stream, c->ev_in, 0));
  }
  void done() {
    HIPCHK(hipEventRecord(c->ev_out, c->stream));
    HIPCHK(hipStreamWaitEvent(user, c->ev_out, 0));
  }
};

// Host checks of an expansion problem; role[o] = 1 for R, 2 for X; occ[o] = 1
// for the occupied orbitals of the reference determinant.
void parse_problem(const mbefci_problem* pb, std::vector<int>& role, std::vector<int>& occ) {
  const int M = pb->norb;
  if (M < 1 || M > kMaxOrb) throw Error(MBEFCI_EINVAL, "norb must be in 1..64");
  if (!pb->h1 || !pb->eri) throw Error(MBEFCI_EINVAL, "null integrals");
  if (pb->nocc < 0 || pb->nref < 0 || pb->nexp < 0 || pb->nocc > M || pb->nref > M ||
      pb->nexp > M)
    throw Error(MBEFCI_EINVAL, "orbital-set sizes out of range");
  if (pb->max_order < 0 || pb->max_order > pb->nexp)
    throw Error(MBEFCI_EINVAL, "max_order must be in 0..nexp");
  role.assign(M, 0);
  occ.assign(M, 0);
  for (int i = 0; i < pb->nocc; ++i) {
    int o = pb->occ[i];
    if (o < 0 || o >= M || occ[o]) throw Error(MBEFCI_EINVAL, "bad occupied orbital list");
    occ[o] = 1;
  }
  for (int i = 0; i < pb->nref; ++i) {
    int o = pb->ref[i];
    if (o < 0 || o >= M || role[o]) throw Error(MBEFCI_EINVAL, "bad reference space");
    role[o] = 1;
  }
  for (int i = 0; i < pb->nexp; ++i) {
    int o = pb->exp[i];
    if (o < 0 || o >= M || role[o])
      throw Error(MBEFCI_EINVAL, "expansion space must be distinct and disjoint from R");
    role[o] = 2;
  }
  if (pb->nref + pb->max_order > 14)
    throw Error(MBEFCI_EUNSUPPORTED, "|R| + max_order exceeds the compiled 14 active orbitals");
  if (pb->orbsym)
    for (int o = 0; o < M; ++o)
      if (pb->orbsym[o] < 0 || pb->orbsym[o] >= kIrreps)
        throw Error(MBEFCI_EINVAL, "orbital irreps must be in 0..7");
}

MbeSpaces make_spaces(int M, const std::vector<int>& role, const std::vector<int>& occ) {
  MbeSpaces sp;
  std::memset(&sp, 0, sizeof(sp));
  sp.M = M;
  for (int o = 0; o < M; ++o) {
    if (role[o] == 1) sp.R[sp.nR++] = o;
    if (role[o] == 2) {
      if (occ[o]) sp.Xo[sp.nXo++] = o;
      else sp.Xv[sp.nXv++] = o;
    }
    if (occ[o]) sp.O[sp.nO++] = o;
    if (role[o] == 1 && occ[o]) ++sp.nocc_ref;
  }
  return sp;
}

// A plan whose construction did not finish is dropped after a failed call.
void discard_partial_plan(mbefci_ctx* c) {
  if (c->plan && !c->plan->ready) {
    if (c->plan->graph) (void)hipGraphExecDestroy(c->plan->graph);
    c->plan.reset();
    c->have_forward = false;
  }
}

template <class F>
int guarded(mbefci_ctx* c, F&& f) {
  if (!c) return MBEFCI_EINVAL;
  try {
    c->err.clear();
    f();
    return MBEFCI_OK;
  } catch (const Error& e) {
    c->err = e.what();
    discard_partial_plan(c);
    return e.code;
  } catch (const std::exception& e) {
    c->err = e.what();
    discard_partial_plan(c);
    return MBEFCI_EDEVICE;
  }
}

void check_shape(int n, int na, int nb) {
  if (n < 0 || n > kMaxActive || na < 0 || nb < 0 || na > n || nb > n)
    throw Error(MBEFCI_EINVAL, "invalid CASCI shape (norb, nalpha, nbeta)");
}

// Build a plan of `nprob` identical-shape CASCIs and fold their Hamiltonians.
void check_orbsym(int n, const int32_t* orbsym, int wfn) {
  if (wfn < 0 || wfn >= kIrreps) throw Error(MBEFCI_EINVAL, "target irrep must be in 0..7");
  for (int t = 0; t < n; ++t)
    if (orbsym[t] < 0 || orbsym[t] >= kIrreps)
      throw Error(MBEFCI_EINVAL, "orbital irreps must be in 0..7");
}

void casci_plan(mbefci_ctx* c, int nprob, int n, int na, int nb, const double* const* h1s,
                const double* const* eris, const double* ecore, const int32_t* orbsym = nullptr,
                int wfn = 0) {
  check_shape(n, na, nb);
  if (n > 14) throw Error(MBEFCI_EUNSUPPORTED, "active space exceeds 14 orbitals");
  if (orbsym) check_orbsym(n, orbsym, wfn);
  if (c->plan && c->plan->graph) HIPCHK(hipGraphExecDestroy(c->plan->graph));
  c->plan.reset(new Plan());
  Plan& P = *c->plan;
  for (int i = 0; i < nprob; ++i) {
    Item I{};
    I.n = n;
    I.na = na;
    I.nb = nb;
    P.items.push_back(I);
  }
  if (orbsym) {
    std::vector<int> os(orbsym, orbsym + n);
    P.item_symtab.assign(nprob, &sym_tab(c, n, na, nb, os.data(), wfn));
  }
  finalize_plan(c, P, c->opts.nguess);
  const double** d_h = arena<const double*>(c, "hptr", nprob);
  const double** d_g = arena<const double*>(c, "gptr", nprob);
  double* d_e = arena<double>(c, "ecore", nprob);
  std::vector<const double*> hv(h1s, h1s + nprob), gv(eris, eris + nprob);
  std::vector<double> ev(ecore, ecore + nprob);
  upload(c, d_h, hv);
  upload(c, d_g, gv);
  upload(c, d_e, ev);
  launch_casci_setup(n, d_h, d_g, d_e, P.d_items, P.nitem, P.hams, P.W, c->stream);
  HIPCHK(hipGetLastError());
  P.ready = true;
}

// ------------------------------------------------------------- RDM pass
// Gamma+ and gamma+ of every multi-determinant CASCI of the plan from the
// CI vectors kept by the last solve (P.ci), into the "rdm" arena
// [item][kpad*kpad] (offsets roff).  Returns the device pointers.
struct RdmOut {
  double* rdmp;
  int64_t* roff;
};

RdmOut rdm_pass(mbefci_ctx* c, Plan& P) {
  if (P.has_sym)
    throw Error(MBEFCI_EUNSUPPORTED, "RDMs of point-group blocked CASCIs are not available");
  const int TN = 64;
  std::vector<std::vector<Work>> gwork(P.groups.size());
  std::vector<int32_t> wlo(P.nitem, 0), whi(P.nitem, 0);
  std::vector<int64_t> roff(P.nitem, 0);
  int64_t rtot = 0;
  for (int i = 0; i < P.nitem; ++i) {
    roff[i] = rtot;
    rtot += (int64_t)P.items[i].kpad * P.items[i].kpad;
  }
  // work units: per beta block, alpha ranges sized so that one CASCI has at
  // most about 512 partials
  std::vector<int> order;  // global work order: group by group, item by item
  std::vector<int64_t> poff;
  int64_t ptot = 0;
  int gcount = 0;
  std::vector<int> wstart(P.groups.size(), 0);
  for (size_t gi = 0; gi < P.groups.size(); ++gi) {
    wstart[gi] = gcount;
    for (int i = 0; i < P.nitem; ++i) {
      if (P.item_group[i] != (int)gi) continue;
      const Item& I = P.items[i];
      const int nblk = (I.Nb + TN - 1) / TN;
      const int csz = std::max(16, (int)(((int64_t)I.Na * nblk + 511) / 512));
      wlo[i] = gcount + (int)gwork[gi].size();
      for (int bk = 0; bk < nblk; ++bk)
        for (int a = 0; a < I.Na; a += csz)
          gwork[gi].push_back(Work{i, bk * I.Na + a, bk * I.Na + std::min(a + csz, I.Na), 0});
      whi[i] = gcount + (int)gwork[gi].size();
    }
    for (size_t k = 0; k < gwork[gi].size(); ++k) {
      poff.push_back(ptot);
      ptot += (int64_t)P.items[gwork[gi][k].item].kpad * P.items[gwork[gi][k].item].kpad;
    }
    gcount += (int)gwork[gi].size();
  }
  double* part = arena<double>(c, "rdm_part", std::max<int64_t>(ptot, 1));
  double* rdmp = arena<double>(c, "rdm", std::max<int64_t>(rtot, 1));
  int64_t* d_roff = arena<int64_t>(c, "rdm_roff", P.nitem);
  int64_t* d_poff = arena<int64_t>(c, "rdm_poff", std::max<size_t>(poff.size(), 1));
  int32_t* d_wlo = arena<int32_t>(c, "rdm_wlo", P.nitem);
  int32_t* d_whi = arena<int32_t>(c, "rdm_whi", P.nitem);
  Work* d_work = arena<Work>(c, "rdm_work", std::max(gcount, 1));
  std::vector<Work> all;
  for (auto& v : gwork) all.insert(all.end(), v.begin(), v.end());
  upload(c, d_roff, roff);
  upload(c, d_poff, poff);
  upload(c, d_wlo, wlo);
  upload(c, d_whi, whi);
  upload(c, d_work, all);
  for (size_t gi = 0; gi < P.groups.size(); ++gi) {
    if (!launch_rdm_syrk(P.groups[gi].n, TN, P.d_items, d_work + wstart[gi],
                         (int)gwork[gi].size(), P.ci, part + (gwork[gi].empty() ? 0 : poff[wstart[gi]]),
                         c->stream))
      throw Error(MBEFCI_EUNSUPPORTED, "no RDM kernel for n=" + std::to_string(P.groups[gi].n));
  }
  launch_rdm_reduce(P.d_items, P.nitem, d_wlo, d_whi, part, d_poff, rdmp, d_roff, c->stream);
  HIPCHK(hipGetLastError());
  return RdmOut{rdmp, d_roff};
}

}  // namespace

// =================================================================== C ABI
namespace {
// Host threads for n independent items: one per 16,384 items, at most 16
// (the host share of one GPU) and at most the hardware's count.
int host_threads(int64_t n) {
  const int hw = std::max(1u, std::thread::hardware_concurrency());
  return (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)16, (int64_t)hw, n / 16384}));
}
// f(t, lo, hi) on nth contiguous chunks of [0, n), chunk 0 on this thread;
// an exception of any chunk is rethrown here after every thread has ended.
template <class F>
void run_chunks(int64_t n, int nth, F f) {
  std::vector<std::thread> pool;
  std::vector<std::exception_ptr> err(nth);
  const int64_t per = (n + nth - 1) / nth;
  auto body = [&f, &err](int t, int64_t lo, int64_t hi) {
    try {
      f(t, lo, hi);
    } catch (...) {
      err[t] = std::current_exception();
    }
  };
  for (int t = 1; t < nth; ++t) {
    const int64_t lo = std::min(n, t * per), hi = std::min(n, lo + per);
    pool.emplace_back(body, t, lo, hi);
  }
  body(0, 0, std::min(n, per));
  for (auto& th : pool) th.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}
// The sorted union of sorted, duplicate-free lists: pairwise merges, each
// round's merges on threads of their own.
std::vector<uint64_t> merge_unique(std::vector<std::vector<uint64_t>>& lists) {
  if (lists.empty()) return {};
  while (lists.size() > 1) {
    const int64_t half = (int64_t)(lists.size() / 2);
    std::vector<std::vector<uint64_t>> out(half + lists.size() % 2);
    run_chunks(half, (int)std::max<int64_t>(1, half), [&](int, int64_t lo, int64_t hi) {
      for (int64_t i = lo; i < hi; ++i) {
        const auto& a = lists[2 * i];
        const auto& b = lists[2 * i + 1];
        std::vector<uint64_t>& m = out[i];
        m.reserve(a.size() + b.size());
        std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(m));
      }
    });
    if (lists.size() % 2) out[half].swap(lists.back());
    lists.swap(out);
  }
  return std::move(lists[0]);
}
}  // namespace

extern "C" {

void mbefci_default_opts(mbefci_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->conv_tol = 1e-6;
  o->max_iter = 200;
  o->max_space = 5;
  o->nguess = 1;
  o->mode = MBEFCI_BATCHED;
  o->use_graph = 1;
  o->tile = 0;
  o->keep_ci = 1;
  o->validate = 1;
  o->sigma_pass_mb = 0;
  o->precond = 0;
  o->pspace = kMaxPspace;
  o->max_workspace = 0;
  o->tune_cache = nullptr;
}

static int check_opts(const mbefci_opts* o, std::string* why) {
  if (!(o->conv_tol > 0)) { *why = "conv_tol must be positive"; return MBEFCI_EINVAL; }
  if (o->max_iter < 1) { *why = "max_iter must be >= 1"; return MBEFCI_EINVAL; }
  if (o->max_space < 3 || o->max_space > kMaxSpace) { *why = "max_space must be in 3..16"; return MBEFCI_EINVAL; }
  if (o->nguess < 1 || o->nguess > 8 || o->nguess + 1 >= o->max_space) { *why = "nguess must be in 1..8 and below max_space - 1"; return MBEFCI_EINVAL; }
  if (o->mode != MBEFCI_BATCHED && o->mode != MBEFCI_PER_LAUNCH) { *why = "unknown mode"; return MBEFCI_EINVAL; }
  if (o->tile != 0 && o->tile != 32 && o->tile != 64 && o->tile != 128) { *why = "tile must be 0, 32, 64 or 128"; return MBEFCI_EINVAL; }
  if (o->sigma_pass_mb < 0) { *why = "sigma_pass_mb must be >= 0"; return MBEFCI_EINVAL; }
  if (o->precond != 0 && o->precond != 1) { *why = "precond must be 0 or 1"; return MBEFCI_EINVAL; }
  if (o->pspace < 0 || o->pspace > kMaxPspace) { *why = "pspace must be in 0..112"; return MBEFCI_EINVAL; }
  if (o->screen_batch < 0) { *why = "screen_batch must be >= 0"; return MBEFCI_EINVAL; }
  return MBEFCI_OK;
}

int mbefci_create(int device, const mbefci_opts* opts, mbefci_ctx** out) {
  if (!out) return MBEFCI_EINVAL;
  *out = nullptr;
  mbefci_opts o;
  mbefci_default_opts(&o);
  if (opts) o = *opts;
  std::string why;
  if (check_opts(&o, &why) != MBEFCI_OK) return MBEFCI_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return MBEFCI_EDEVICE;
  }
  auto* c = new mbefci_ctx();
  c->device = device;
  c->opts = o;
  if (hipSetDevice(device) != hipSuccess ||
      hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess ||
      hipEventCreate(&c->t0) != hipSuccess || hipEventCreate(&c->t1) != hipSuccess) {
    delete c;
    return MBEFCI_EDEVICE;
  }
  // device address of the no-allocation sigma's scratch array on this device;
  // a failure is reported by mbefci_sigma_noalloc, which tries again
  if (mbefci::noalloc_init(device) != hipSuccess) (void)hipGetLastError();
  *out = c;
  return MBEFCI_OK;
}

void mbefci_destroy(mbefci_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->plan && c->plan->graph) (void)hipGraphExecDestroy(c->plan->graph);
  for (auto& kv : c->tabs) {
    if (kv.second.link) (void)hipFree(kv.second.link);
    if (kv.second.linkT) (void)hipFree(kv.second.linkT);
    if (kv.second.str) (void)hipFree(kv.second.str);
    if (kv.second.pair) (void)hipFree(kv.second.pair);
    if (kv.second.pairT) (void)hipFree(kv.second.pairT);
  }
  for (auto& kv : c->symtabs)
    if (kv.second.block) (void)hipFree(kv.second.block);
  for (auto& kv : c->bufs) release_buf(c, kv.second);
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  if (c->t0) (void)hipEventDestroy(c->t0);
  if (c->t1) (void)hipEventDestroy(c->t1);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* mbefci_last_error(const mbefci_ctx* c) { return c ? c->err.c_str() : "null context"; }

int mbefci_set_allocator(mbefci_ctx* c, void* (*alloc)(size_t, void*),
                         void (*release)(void*, void*), void* user) {
  if (!c) return MBEFCI_EINVAL;
  if ((alloc == nullptr) != (release == nullptr)) {
    c->err = "set_allocator needs both functions or neither";
    return MBEFCI_EINVAL;
  }
  return guarded(c, [&] {
    HIPCHK(hipSetDevice(c->device));
    // every workspace block goes back to the allocator it came from; the
    // cached plan and the kept CI vectors go with them
    if (c->plan && c->plan->graph) HIPCHK(hipGraphExecDestroy(c->plan->graph));
    c->plan.reset();
    c->have_forward = false;
    for (auto& kv : c->bufs) release_buf(c, kv.second);
    c->bufs.clear();
    c->alloc_fn = alloc;
    c->release_fn = release;
    c->alloc_user = user;
  });
}

int mbefci_set_opts(mbefci_ctx* c, const mbefci_opts* o) {
  if (!c || !o) return MBEFCI_EINVAL;
  std::string why;
  int rc = check_opts(o, &why);
  if (rc != MBEFCI_OK) {
    c->err = why;
    return rc;
  }
  bool plan_dead = o->max_space != c->opts.max_space || o->tile != c->opts.tile ||
                   o->sigma_pass_mb != c->opts.sigma_pass_mb || o->precond != c->opts.precond ||
                   o->pspace != c->opts.pspace;
  // the captured iteration graph holds the tolerance and the iteration cap
  // as kernel arguments: it is captured again at the next solve
  const bool graph_dead = o->conv_tol != c->opts.conv_tol || o->max_iter != c->opts.max_iter;
  c->opts = *o;
  if (plan_dead && c->plan) {
    if (c->plan->graph) (void)hipGraphExecDestroy(c->plan->graph);
    c->plan.reset();
    c->have_forward = false;
  } else if (graph_dead && c->plan && c->plan->graph) {
    (void)hipGraphExecDestroy(c->plan->graph);
    c->plan->graph = nullptr;
  }
  return MBEFCI_OK;
}

int64_t mbefci_num_strings(int32_t norb, int32_t nelec) {
  if (norb < 0 || norb > 64 || nelec < 0 || nelec > norb) return 0;
  return binom_host(norb, nelec);
}
int32_t mbefci_num_links(int32_t norb, int32_t nelec) {
  if (norb < 0 || norb > 64 || nelec < 0 || nelec > norb) return 0;
  return nelec * (norb - nelec + 1);
}
int64_t mbefci_num_tuples(int32_t nexp, int32_t max_order) {
  if (nexp < 0 || max_order < 0 || max_order > nexp || nexp > 64) return 0;
  int64_t s = 0;
  for (int n = 1; n <= max_order; ++n) s += binom_host(nexp, n);
  return s;
}

// ---- integer layer on the host (no context, no device) -----------------------
namespace {
// Strings of nelec electrons in norb orbitals in ascending integer order: the
// next larger integer with the same number of set bits (Gosper's method).
// Returns false when the count exceeds the int32 addresses of the tables.
bool host_strings(int norb, int nelec, std::vector<uint64_t>* out) {
  const int64_t N = binom_host(norb, nelec);
  if (N <= 0 || N > INT32_MAX) return false;
  out->resize(N);
  uint64_t v = nelec == 64 ? ~(uint64_t)0 : (((uint64_t)1 << nelec) - 1);
  for (int64_t i = 0; i < N; ++i) {
    (*out)[i] = v;
    if (i + 1 < N) {
      const uint64_t t = v | (v - 1);
      v = (t + 1) | (((~t & (t + 1)) - 1) >> (__builtin_ctzll(v) + 1));
    }
  }
  return true;
}
// address = sum_j C(o_j, j) over the occupied orbitals o_1 < o_2 < ...
int64_t host_string_addr(uint64_t m) {
  int64_t a = 0;
  int j = 1;
  for (; m; m &= m - 1, ++j) a += binom_host(__builtin_ctzll(m), j);
  return a;
}
}  // namespace

int mbefci_strings(int32_t norb, int32_t nelec, uint64_t* out) {
  if (norb < 0 || norb > 64 || nelec < 0 || nelec > norb || !out) return MBEFCI_EINVAL;
  try {
    std::vector<uint64_t> s;
    if (!host_strings(norb, nelec, &s)) return MBEFCI_EINVAL;
    std::copy(s.begin(), s.end(), out);
    return MBEFCI_OK;
  } catch (const std::exception&) {
    return MBEFCI_ENOMEM;
  }
}

int mbefci_link_table(int32_t norb, int32_t nelec, int32_t* out) {
  if (norb < 0 || norb > 32 || nelec < 0 || nelec > norb || !out) return MBEFCI_EINVAL;
  try {
    std::vector<uint64_t> s;
    if (!host_strings(norb, nelec, &s)) return MBEFCI_EINVAL;
    const int64_t L = (int64_t)nelec * (norb - nelec + 1);
    for (size_t I = 0; I < s.size(); ++I) {
      const uint64_t m = s[I];
      int32_t* e = out + (int64_t)I * L * 4;
      int idx = 0;
      for (int o = 0; o < norb; ++o)  // E_oo I = I for occupied o
        if (m >> o & 1) {
          e[4 * idx] = o, e[4 * idx + 1] = o, e[4 * idx + 2] = (int32_t)I, e[4 * idx + 3] = 1;
          ++idx;
        }
      for (int q = 0; q < norb; ++q) {
        if (!(m >> q & 1)) continue;
        for (int p = 0; p < norb; ++p) {
          if (m >> p & 1) continue;
          const uint64_t r = (m & ~((uint64_t)1 << q)) | ((uint64_t)1 << p);
          const int lo = std::min(p, q), hi = std::max(p, q);
          const uint64_t between = (((uint64_t)1 << hi) - 1) & ~((((uint64_t)1 << lo) << 1) - 1);
          e[4 * idx] = p;
          e[4 * idx + 1] = q;
          e[4 * idx + 2] = (int32_t)host_string_addr(r);
          e[4 * idx + 3] = (__builtin_popcountll(m & between) & 1) ? -1 : 1;
          ++idx;
        }
      }
    }
    return MBEFCI_OK;
  } catch (const std::exception&) {
    return MBEFCI_ENOMEM;
  }
}

int mbefci_strings_device(mbefci_ctx* c, int32_t norb, int32_t nelec, uint64_t* out,
                          void* stream) {
  return guarded(c, [&] {
    if (norb < 0 || norb > 64 || nelec < 0 || nelec > norb || !out)
      throw Error(MBEFCI_EINVAL, "invalid string shape");
    StreamScope sc(c, stream);
    launch_strings(norb, nelec, binom_host(norb, nelec), out, c->stream);
    HIPCHK(hipGetLastError());
    sc.done();
  });
}

int mbefci_link_table_device(mbefci_ctx* c, int32_t norb, int32_t nelec, int32_t* out,
                             void* stream) {
  return guarded(c, [&] {
    if (norb < 0 || norb > 32 || nelec < 0 || nelec > norb || !out)
      throw Error(MBEFCI_EINVAL, "invalid link-table shape");
    StreamScope sc(c, stream);
    launch_links(norb, nelec, binom_host(norb, nelec), nullptr, nullptr, out, c->stream);
    HIPCHK(hipGetLastError());
    sc.done();
  });
}

int mbefci_hdiag(mbefci_ctx* c, int32_t n, int32_t na, int32_t nb, const double* h1,
                 const double* eri, double e_core, double* diag, void* stream) {
  return guarded(c, [&] {
    check_shape(n, na, nb);
    if (!h1 || !eri || !diag) throw Error(MBEFCI_EINVAL, "null pointer");
    StreamScope sc(c, stream);
    check_integrals(c, n, h1, eri);
    casci_plan(c, 1, n, na, nb, &h1, &eri, &e_core);
    Plan& P = *c->plan;
    launch_hdiag(P.d_items, P.d_blocks, P.nblock, P.hams, P.diag, c->stream);
    launch_add_scalar(diag, P.diag, e_core, P.items[0].ndet, c->stream);
    HIPCHK(hipGetLastError());
    c->have_forward = false;
    sc.done();
  });
}

int mbefci_sigma(mbefci_ctx* c, int32_t n, int32_t na, int32_t nb, const double* h1,
                 const double* eri, double e_core, const double* cvec, double* sig, void* stream) {
  return guarded(c, [&] {
    check_shape(n, na, nb);
    if (!h1 || !eri || !cvec || !sig) throw Error(MBEFCI_EINVAL, "null pointer");
    StreamScope sc(c, stream);
    check_integrals(c, n, h1, eri);
    casci_plan(c, 1, n, na, nb, &h1, &eri, &e_core);
    Plan& P = *c->plan;
    const int64_t nd = P.items[0].ndet;
    if (nd > 1) {
      HIPCHK(hipMemcpyAsync(P.V, cvec, nd * 8, hipMemcpyDeviceToDevice, c->stream));
      launch_state_single(P.st, c->stream);
      sigma(c, P, whole(P), 0);
      // e_core c is added here; the folded one- and two-body part is in S
      launch_axpy_out(sig, P.S, cvec, e_core, nd, c->stream);
    } else {
      // a single determinant: sigma = H_00 c
      launch_hdiag(P.d_items, P.d_blocks, P.nblock, P.hams, P.diag, c->stream);
      launch_diag_times(sig, P.diag, cvec, e_core, 1, c->stream);
    }
    HIPCHK(hipGetLastError());
    c->have_forward = false;
    sc.done();
  });
}

int mbefci_sigma_noalloc(mbefci_ctx* c, int32_t n, int32_t na, int32_t nb, const double* h1,
                         const double* eri, double e_core, const double* cvec, double* sig,
                         void* stream) {
  if (!c) return MBEFCI_EINVAL;
  c->err.clear();
  const hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) {
    c->err = std::string("hipSetDevice: ") + hipGetErrorString(e);
    return MBEFCI_EDEVICE;
  }
  std::string why;
  const int rc = mbefci::noalloc_sigma(c->device, n, na, nb, h1, eri, e_core, cvec, sig,
                                       (hipStream_t)stream, &why);
  if (rc != MBEFCI_OK) c->err = why;
  return rc;
}

namespace {
// Solve a batch of same-shape CASCIs (the caller's StreamScope is active);
// copies the CI vectors to ci_out[i] when given (needs keep_ci).
void casci_batch(mbefci_ctx* c, int32_t nprob, int32_t n, int32_t na, int32_t nb,
                 const double* const* h1s, const double* const* eris, const double* e_core,
                 double* e_out, double* const* ci_out, mbefci_stats* stats,
                 const int32_t* orbsym = nullptr, int wfn = 0) {
  auto t_start = std::chrono::steady_clock::now();
  check_shape(n, na, nb);
  if (nprob < 1 || !h1s || !eris || !e_core || !e_out)
    throw Error(MBEFCI_EINVAL, "invalid batch arguments");
  bool want_ci = false;
  for (int i = 0; ci_out && i < nprob; ++i) want_ci |= ci_out[i] != nullptr;
  if (want_ci && !c->opts.keep_ci)
    throw Error(MBEFCI_EINVAL, "CI vectors requested with keep_ci = 0");
  for (int i = 0; i < nprob; ++i) {
    if (!h1s[i] || !eris[i]) throw Error(MBEFCI_EINVAL, "null integral pointer");
    check_integrals(c, n, h1s[i], eris[i]);
  }
  casci_plan(c, nprob, n, na, nb, h1s, eris, e_core, orbsym, wfn);
  Plan& P = *c->plan;
  mbefci_stats st{};
  solve_plan(c, P, &st);
  launch_item_energy(P.d_items, P.hams, P.st, P.nitem, P.f, c->stream);
  std::vector<double> e(nprob);
  HIPCHK(hipMemcpyAsync(e.data(), P.f, nprob * 8, hipMemcpyDeviceToHost, c->stream));
  if (want_ci)
    for (int i = 0; i < nprob; ++i)
      if (ci_out[i])
        HIPCHK(hipMemcpyAsync(ci_out[i], P.ci + P.items[i].off, P.items[i].ndet * 8,
                              hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  std::copy(e.begin(), e.end(), e_out);
  c->have_forward = true;
  st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                          t_start).count();
  if (stats) *stats = st;
}

// RDMs of the CI vectors kept by the last casci_batch (StreamScope active).
void casci_rdms(mbefci_ctx* c, double* const* rdm1s, double* const* rdm2s) {
  if (!c->plan || c->plan->is_mbe || !c->have_forward)
    throw Error(MBEFCI_EINVAL, "the RDMs need a preceding CASCI solve on ctx");
  if (!c->opts.keep_ci) throw Error(MBEFCI_EINVAL, "CI vectors were not kept (keep_ci = 0)");
  Plan& P = *c->plan;
  RdmOut R = rdm_pass(c, P);
  for (int i = 0; i < P.nitem; ++i)
    launch_casci_rdm_out(P.d_items, i, P.items[i].n, R.rdmp, R.roff, rdm1s ? rdm1s[i] : nullptr,
                         rdm2s ? rdm2s[i] : nullptr, c->stream);
  HIPCHK(hipGetLastError());
}
}  // namespace

int mbefci_casci_batch(mbefci_ctx* c, int32_t nprob, int32_t n, int32_t na, int32_t nb,
                       const double* const* h1s, const double* const* eris, const double* e_core,
                       double* e_out, double* const* ci_out, mbefci_stats* stats, void* stream) {
  return guarded(c, [&] {
    StreamScope sc(c, stream);
    casci_batch(c, nprob, n, na, nb, h1s, eris, e_core, e_out, ci_out, stats);
    sc.done();
  });
}

int mbefci_casci(mbefci_ctx* c, int32_t n, int32_t na, int32_t nb, const double* h1,
                 const double* eri, double e_core, double* e_out, double* ci_out, double* rdm1,
                 double* rdm2, void* stream) {
  return guarded(c, [&] {
    if (!c->opts.keep_ci && (ci_out || rdm1 || rdm2))
      throw Error(MBEFCI_EINVAL, "CI vector or RDMs requested with keep_ci = 0");
    StreamScope sc(c, stream);
    double* const cis[1] = {ci_out};
    casci_batch(c, 1, n, na, nb, &h1, &eri, &e_core, e_out, ci_out ? cis : nullptr, nullptr);
    if (rdm1 || rdm2) {
      double* const r1[1] = {rdm1};
      double* const r2[1] = {rdm2};
      casci_rdms(c, r1, r2);
    }
    sc.done();
  });
}

int mbefci_casci_rdm(mbefci_ctx* c, double* const* rdm1s, double* const* rdm2s, void* stream) {
  return guarded(c, [&] {
    StreamScope sc(c, stream);
    casci_rdms(c, rdm1s, rdm2s);
    sc.done();
  });
}

int64_t mbefci_sym_ndet(int32_t norb, int32_t nalpha, int32_t nbeta, const int32_t* orbsym,
                        int32_t wfnsym) {
  if (norb < 0 || norb > 64 || nalpha < 0 || nbeta < 0 || nalpha > norb || nbeta > norb ||
      !orbsym || wfnsym < 0 || wfnsym >= kIrreps)
    return MBEFCI_EINVAL;
  for (int t = 0; t < norb; ++t)
    if (orbsym[t] < 0 || orbsym[t] >= kIrreps) return MBEFCI_EINVAL;
  // strings per irrep, by dynamic programming over the orbitals
  auto count = [&](int ne, int64_t* out) {
    std::vector<std::array<int64_t, kIrreps>> dp(ne + 1);
    for (auto& r : dp) r.fill(0);
    dp[0][0] = 1;
    for (int t = 0; t < norb; ++t)
      for (int k = std::min(ne, t + 1); k >= 1; --k)
        for (int a = 0; a < kIrreps; ++a) dp[k][a ^ orbsym[t]] += dp[k - 1][a];
    for (int a = 0; a < kIrreps; ++a) out[a] = dp[ne][a];
  };
  int64_t A[kIrreps], B[kIrreps];
  count(nalpha, A);
  count(nbeta, B);
  int64_t nd = 0;
  for (int a = 0; a < kIrreps; ++a) nd += A[a] * B[a ^ wfnsym];
  return nd;
}

int mbefci_casci_sym(mbefci_ctx* c, int32_t nprob, int32_t n, int32_t na, int32_t nb,
                     const int32_t* orbsym, int32_t wfnsym, const double* const* h1s,
                     const double* const* eris, const double* e_core, double* e_out,
                     double* const* ci_out, mbefci_stats* stats, void* stream) {
  return guarded(c, [&] {
    if (!orbsym) throw Error(MBEFCI_EINVAL, "null orbital irreps");
    StreamScope sc(c, stream);
    casci_batch(c, nprob, n, na, nb, h1s, eris, e_core, e_out, ci_out, stats, orbsym, wfnsym);
    sc.done();
  });
}

int mbefci_sigma_sym(mbefci_ctx* c, int32_t n, int32_t na, int32_t nb, const int32_t* orbsym,
                     int32_t wfnsym, const double* h1, const double* eri, double e_core,
                     const double* cvec, double* sig, void* stream) {
  return guarded(c, [&] {
    check_shape(n, na, nb);
    if (!h1 || !eri || !cvec || !sig || !orbsym) throw Error(MBEFCI_EINVAL, "null pointer");
    StreamScope sc(c, stream);
    check_integrals(c, n, h1, eri);
    casci_plan(c, 1, n, na, nb, &h1, &eri, &e_core, orbsym, wfnsym);
    Plan& P = *c->plan;
    const int64_t nd = P.items[0].ndet;
    if (nd > 1) {
      HIPCHK(hipMemcpyAsync(P.V, cvec, nd * 8, hipMemcpyDeviceToDevice, c->stream));
      launch_state_single(P.st, c->stream);
      sigma(c, P, whole(P), 0);
      launch_axpy_out(sig, P.S, cvec, e_core, nd, c->stream);
    } else {
      launch_hdiag(P.d_items, P.d_blocks, P.nblock, P.hams, P.diag, c->stream);
      launch_diag_times(sig, P.diag, cvec, e_core, 1, c->stream);
    }
    HIPCHK(hipGetLastError());
    c->have_forward = false;
    sc.done();
  });
}

int mbefci_mbe_forward(mbefci_ctx* c, const mbefci_problem* pb, double* e_ref, double* e_order,
                       double* e_total, double* tuple_incr, double* tuple_energy,
                       mbefci_stats* stats, void* stream) {
  return guarded(c, [&] {
    auto t_start = std::chrono::steady_clock::now();
    if (!pb || !e_ref || !e_total || (pb->max_order > 0 && !e_order))
      throw Error(MBEFCI_EINVAL, "null argument");
    const int M = pb->norb;
    std::vector<int> role, occ;
    parse_problem(pb, role, occ);
    if (pb->orbsym)
      throw Error(MBEFCI_EUNSUPPORTED, "orbital irreps: use mbefci_mbe_screened (t_init = 0 "
                                       "gives the full expansion)");
    StreamScope sc(c, stream);
    check_integrals(c, M, pb->h1, pb->eri);

    // ---- plan (bucket by order and occupied count; items in bucket order)
    std::string sig = std::to_string(M) + "|" + std::to_string(pb->max_order) + "|";
    for (int i = 0; i < M; ++i) sig += char('0' + role[i] + 3 * occ[i]);
    const bool reuse = c->plan && c->plan->ready && c->plan->is_mbe && c->plan->signature == sig;
    if (!reuse) {
      if (c->plan && c->plan->graph) HIPCHK(hipGraphExecDestroy(c->plan->graph));
      c->plan.reset(new Plan());
      Plan& P = *c->plan;
      P.is_mbe = true;
      P.signature = sig;
      P.max_order = pb->max_order;
      P.norb = M;
      MbeSpaces& sp = P.sp;
      std::memset(&sp, 0, sizeof(sp));
      sp.M = M;
      std::vector<int> R, Xo, Xv, O;
      for (int o = 0; o < M; ++o) {
        if (role[o] == 1) R.push_back(o);
        if (role[o] == 2) (occ[o] ? Xo : Xv).push_back(o);
        if (occ[o]) O.push_back(o);
      }
      sp.nR = (int)R.size();
      sp.nXo = (int)Xo.size();
      sp.nXv = (int)Xv.size();
      sp.nO = (int)O.size();
      std::copy(R.begin(), R.end(), sp.R);
      std::copy(Xo.begin(), Xo.end(), sp.Xo);
      std::copy(Xv.begin(), Xv.end(), sp.Xv);
      std::copy(O.begin(), O.end(), sp.O);
      int nref_occ = 0;
      for (int o : R) nref_occ += occ[o];
      sp.nocc_ref = nref_occ;
      P.buckets.push_back(BucketDev{0, 0, 0, 1});
      {
        Item I{};
        I.n = sp.nR;
        I.na = I.nb = nref_occ;
        P.items.push_back(I);
      }
      for (int n = 1; n <= pb->max_order; ++n)
        for (int a = 0; a <= n; ++a) {
          int64_t cnt = binom_host(sp.nXo, a) * binom_host(sp.nXv, n - a);
          if (cnt == 0) continue;
          P.buckets.push_back(BucketDev{n, a, (int64_t)P.items.size(), cnt});
          for (int64_t k = 0; k < cnt; ++k) {
            Item I{};
            I.n = sp.nR + n;
            I.na = I.nb = nref_occ + a;
            P.items.push_back(I);
          }
        }
      P.ntuples = (int64_t)P.items.size() - 1;
      finalize_plan(c, P, c->opts.nguess);
      P.d_buckets = arena<BucketDev>(c, "buckets", P.buckets.size());
      upload(c, P.d_buckets, P.buckets);
      P.tuple_pos = arena<int32_t>(c, "tuple_pos", (size_t)P.nitem * (2 * P.max_order + 2));
      P.act = arena<int32_t>(c, "act", (size_t)P.nitem * kMaxActive);
      // X sorted; positions of Xo / Xv members in it (for lexicographic output)
      std::vector<int> xs;
      for (int o = 0; o < M; ++o)
        if (role[o] == 2) xs.push_back(o);
      P.xsorted = xs;
      std::vector<int32_t> po(std::max(1, sp.nXo)), pv(std::max(1, sp.nXv));
      for (int i = 0; i < sp.nXo; ++i)
        po[i] = (int32_t)(std::find(xs.begin(), xs.end(), Xo[i]) - xs.begin());
      for (int i = 0; i < sp.nXv; ++i)
        pv[i] = (int32_t)(std::find(xs.begin(), xs.end(), Xv[i]) - xs.begin());
      int32_t* d_po = arena<int32_t>(c, "xpos_o", po.size());
      int32_t* d_pv = arena<int32_t>(c, "xpos_v", pv.size());
      upload(c, d_po, po);
      upload(c, d_pv, pv);
      std::vector<int64_t> ooff(std::max(1, P.max_order));
      int64_t acc = 0;
      for (int n = 1; n <= P.max_order; ++n) {
        ooff[n - 1] = acc;
        acc += binom_host((int)xs.size(), n);
      }
      int64_t* d_oo = arena<int64_t>(c, "order_off", ooff.size());
      upload(c, d_oo, ooff);
    }
    Plan& P = *c->plan;
    P.ready = true;
    c->have_forward = false;  // until this solve has succeeded
    // ---- set-up, solve, combine
    launch_mbe_setup(&P.sp, P.d_buckets, (int)P.buckets.size(), P.d_items, P.nitem, pb->h1,
                     pb->eri, pb->e_const, P.hams, P.W, P.tuple_pos, P.max_order, P.act, c->stream);
    HIPCHK(hipGetLastError());
    mbefci_stats st{};
    solve_plan(c, P, &st);
    launch_item_energy(P.d_items, P.hams, P.st, P.nitem, P.f, c->stream);
    double* d_lex = arena<double>(c, "inc_lex", std::max<int64_t>(P.ntuples, 1));
    double* d_flex = arena<double>(c, "f_lex", std::max<int64_t>(P.ntuples, 1));
    double* d_eord = arena<double>(c, "e_order", std::max(P.max_order, 1));
    double* d_tot = arena<double>(c, "e_tot", 2);
    launch_mbe_combine(&P.sp, P.d_buckets, (int)P.buckets.size(), P.tuple_pos, P.max_order, P.f,
                       P.nitem, P.inc, d_lex, d_flex,
                       static_cast<int64_t*>(c->bufs["order_off"].p),
                       static_cast<int32_t*>(c->bufs["xpos_o"].p),
                       static_cast<int32_t*>(c->bufs["xpos_v"].p), (int)P.xsorted.size(), d_eord,
                       c->stream);
    launch_mbe_total(P.f, d_eord, P.max_order, d_tot, c->stream);
    HIPCHK(hipGetLastError());
    double tot[2];
    std::vector<double> eo(std::max(P.max_order, 1));
    HIPCHK(hipMemcpyAsync(tot, d_tot, 16, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(eo.data(), d_eord, eo.size() * 8, hipMemcpyDeviceToHost, c->stream));
    std::vector<double> lex, flex;
    if (tuple_incr && P.ntuples > 0) {
      lex.resize(P.ntuples);
      HIPCHK(hipMemcpyAsync(lex.data(), d_lex, P.ntuples * 8, hipMemcpyDeviceToHost, c->stream));
    }
    if (tuple_energy && P.ntuples > 0) {
      flex.resize(P.ntuples);
      HIPCHK(hipMemcpyAsync(flex.data(), d_flex, P.ntuples * 8, hipMemcpyDeviceToHost,
                            c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    *e_ref = tot[0];
    *e_total = tot[1];
    for (int n = 0; n < P.max_order; ++n) e_order[n] = eo[n];
    if (tuple_incr && P.ntuples > 0) std::copy(lex.begin(), lex.end(), tuple_incr);
    if (tuple_energy && P.ntuples > 0) std::copy(flex.begin(), flex.end(), tuple_energy);
    c->have_forward = true;
    st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                            t_start).count();
    if (stats) *stats = st;
    sc.done();
  });
}

int mbefci_partition(int32_t type, int32_t norb, int32_t nocc, const int32_t* occ, int32_t* ref,
                     int32_t* nref, int32_t* exp, int32_t* nexp) {
  if (type < MBEFCI_TYPE1 || type > MBEFCI_TYPE3 || norb < 1 || norb > kMaxOrb || nocc < 0 ||
      nocc > norb || (nocc > 0 && !occ) || !ref || !nref || !exp || !nexp)
    return MBEFCI_EINVAL;
  std::vector<int> is_occ(norb, 0);
  for (int i = 0; i < nocc; ++i) {
    if (occ[i] < 0 || occ[i] >= norb || is_occ[occ[i]]) return MBEFCI_EINVAL;
    is_occ[occ[i]] = 1;
  }
  int nr = 0, nx = 0;
  for (int p = 0; p < norb; ++p) {
    bool in_ref = false;
    if (type == MBEFCI_TYPE1) in_ref = !is_occ[p];
    if (type == MBEFCI_TYPE2) in_ref = is_occ[p] != 0;
    if (in_ref) ref[nr++] = p;
    else exp[nx++] = p;
  }
  *nref = nr;
  *nexp = nx;
  return MBEFCI_OK;
}

int mbefci_mbe_screened(mbefci_ctx* c, const mbefci_problem* pb, const mbefci_screen* scr,
                        double* e_ref, double* e_order, double* e_total, int64_t* n_order,
                        mbefci_stats* stats, void* stream) {
  return guarded(c, [&] {
    auto t_start = std::chrono::steady_clock::now();
    if (!pb || !scr || !e_ref || !e_total || (pb->max_order > 0 && (!e_order || !n_order)))
      throw Error(MBEFCI_EINVAL, "null argument");
    std::vector<int> role, occ;
    parse_problem(pb, role, occ);
    if (!(scr->t_init >= 0.0) || !std::isfinite(scr->t_init) || !(scr->a >= 1.0) ||
        !std::isfinite(scr->a) || scr->m_init < 0)
      throw Error(MBEFCI_EINVAL, "screening needs t_init >= 0, a >= 1 and m_init >= 0");
    const int M = pb->norb, K = pb->max_order;
    StreamScope sc(c, stream);
    check_integrals(c, M, pb->h1, pb->eri);
    // every order gets a plan of its own; the cached expansion plan is dropped
    if (c->plan && c->plan->graph) HIPCHK(hipGraphExecDestroy(c->plan->graph));
    c->plan.reset();
    c->have_forward = false;
    const MbeSpaces sp = make_spaces(M, role, occ);
    std::vector<int> xs;
    uint64_t occx = 0;
    for (int o = 0; o < M; ++o)
      if (role[o] == 2) {
        xs.push_back(o);
        if (occ[o]) occx |= (uint64_t)1 << o;
      }
    const bool vacuum = sp.nR == 0;
    // Eq. 3: with no reference space, tuples of only occupied or only virtual
    // MOs have vanishing increments by construction; they are not computed
    auto structural = [&](uint64_t m) {
      if (!vacuum) return false;
      const int o = __builtin_popcountll(m & occx);
      return o == 0 || o == __builtin_popcountll(m);
    };
    // Eq. 4
    auto threshold = [&](uint64_t m) {
      const int o = __builtin_popcountll(m & occx), v = __builtin_popcountll(m) - o;
      const int mt = std::max(o, v);
      return mt < scr->m_init ? 0.0 : scr->t_init * std::pow(scr->a, (double)(mt - scr->m_init));
    };
    // determinants of the CASCI of tuple m: C(n, na)^2
    auto tuple_dets = [&](uint64_t m) {
      const int n = sp.nR + __builtin_popcountll(m);
      const int na = sp.nocc_ref + __builtin_popcountll(m & occx);
      int64_t b = 1;
      for (int i = 1; i <= na; ++i) b = b * (n - na + i) / i;
      return b * b;
    };
    c->scr_masks.assign(K + 1, {});
    c->scr_inc.assign(K + 1, {});
    for (int k = 0; k < K; ++k) n_order[k] = 0;
    ScreenArrays lower{};
    double* d_eref = arena<double>(c, "scr_eref", 1);
    double* d_eord = arena<double>(c, "scr_eord", std::max(K, 1));
    double* d_tot = arena<double>(c, "scr_tot", 2);
    launch_fill(d_eord, std::max(K, 1), 0.0, c->stream);
    // first level: order 1, or with no reference space the mixed pairs
    int k = 1;
    std::vector<uint64_t> level;
    for (int p : xs)
      if (!structural((uint64_t)1 << p)) level.push_back((uint64_t)1 << p);
    if (level.empty() && vacuum) {
      k = 2;
      for (size_t i = 0; i < xs.size(); ++i)
        for (size_t j = i + 1; j < xs.size(); ++j) {
          const uint64_t m = ((uint64_t)1 << xs[i]) | ((uint64_t)1 << xs[j]);
          if (!structural(m)) level.push_back(m);
        }
    }
    mbefci_stats tot{};
    tot.first_failed = -1;
    bool first = true;
    for (;;) {
      const bool run = k <= K && !level.empty();
      if (!run && !first) break;
      if (!std::is_sorted(level.begin(), level.end())) std::sort(level.begin(), level.end());
      level.erase(std::unique(level.begin(), level.end()), level.end());
      // the order's tuples are solved in chunks of bounded size (items and
      // determinants), so that an order of any width fits the device; their
      // energies f(T) land in one order-wide array
      const int64_t n = run ? (int64_t)level.size() : 0;
      double* d_f = arena<double>(c, "scr_f", std::max<int64_t>(n, 1));
      int64_t lo = 0;
      do {
        std::vector<uint64_t> masks;
        const bool with_ref = first;
        if (with_ref) masks.push_back(0);  // the reference CASCI (E_ref)
        const int64_t max_items = c->opts.screen_batch > 0 ? c->opts.screen_batch
                                                           : kScreenChunkItems;
        int64_t hi = lo, dets = 0;
        while (hi < n && (hi == lo || ((int64_t)masks.size() < max_items &&
                                       dets + tuple_dets(level[hi]) <= kScreenChunkDets))) {
          dets += tuple_dets(level[hi]);
          masks.push_back(level[hi++]);
        }
        if (c->plan && c->plan->graph) HIPCHK(hipGraphExecDestroy(c->plan->graph));
        c->plan.reset(new Plan());
        Plan& P = *c->plan;
        P.norb = M;
        P.sp = sp;
        for (uint64_t m : masks) {
          Item I{};
          I.n = sp.nR + __builtin_popcountll(m);
          I.na = I.nb = sp.nocc_ref + __builtin_popcountll(m & occx);
          P.items.push_back(I);
          if (pb->orbsym) {
            // point-group blocked CASCI in the irrep of the closed-shell
            // reference determinant (totally symmetric); active orbitals
            // ascending, as the set-up kernel takes them
            uint64_t a = m;
            for (int r = 0; r < sp.nR; ++r) a |= (uint64_t)1 << sp.R[r];
            int os[kMaxActive];
            int t = 0;
            for (uint64_t x = a; x; x &= x - 1) os[t++] = pb->orbsym[__builtin_ctzll(x)];
            P.item_symtab.push_back(&sym_tab(c, I.n, I.na, I.nb, os, 0));
          }
        }
        finalize_plan(c, P, c->opts.nguess);
        uint64_t* d_masks = arena<uint64_t>(c, "scr_items", masks.size());
        upload(c, d_masks, masks);
        launch_mbe_setup_list(&P.sp, d_masks, P.d_items, P.nitem, pb->h1, pb->eri, pb->e_const,
                              P.hams, P.W, c->stream);
        HIPCHK(hipGetLastError());
        P.ready = true;
        mbefci_stats st{};
        solve_plan(c, P, &st);
        tot.ntuples += st.ntuples - (with_ref ? 1 : 0);
        tot.nsingle += st.nsingle;
        tot.sigma_calls += st.sigma_calls;
        tot.ndet_total += st.ndet_total;
        tot.max_iters = std::max(tot.max_iters, st.max_iters);
        tot.nbuckets += st.nbuckets;
        tot.graph_launches += st.graph_launches;
        tot.ms_solve += st.ms_solve;
        launch_item_energy(P.d_items, P.hams, P.st, P.nitem, P.f, c->stream);
        const int off = with_ref ? 1 : 0;
        if (with_ref) {
          HIPCHK(hipMemcpyAsync(d_eref, P.f, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
          first = false;
        }
        if (hi > lo)
          HIPCHK(hipMemcpyAsync(d_f + lo, P.f + off, (hi - lo) * sizeof(double),
                                hipMemcpyDeviceToDevice, c->stream));
        lo = hi;
      } while (lo < n);
      if (!run) break;
      uint64_t* dm = arena<uint64_t>(c, "scr_mask" + std::to_string(k), n);
      double* di = arena<double>(c, "scr_inc" + std::to_string(k), n);
      upload(c, dm, level);
      launch_screen_increments(dm, n, k, d_f, d_eref, lower, di, d_eord + (k - 1), c->stream);
      HIPCHK(hipGetLastError());
      lower.mask[k] = dm;
      lower.inc[k] = di;
      lower.n[k] = n;
      std::vector<double> inc(n);
      HIPCHK(hipMemcpyAsync(inc.data(), di, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      n_order[k - 1] = n;
      c->scr_masks[k] = level;
      c->scr_inc[k] = inc;
      if (k == K) break;
      // spawn order k+1 (the per-parent rule with Eq. 4): a computed parent P
      // and a candidate orbital c outside it spawn P + c when one of the
      // order-k tuples S + c (S a (k-1)-subtuple of P, so never P itself) was
      // computed with |Delta eps| above its own threshold.  Over all parents
      // this is: the child has a significant order-k sub-tuple Q and a
      // second computed one (the parent P != Q).  Candidates come from the
      // significant tuples; each keeps its place if at least two of its
      // order-k sub-tuples were computed.  `level` is sorted.
      // Host threads (at most 16) take contiguous chunks of the parents, then
      // of the candidates; the result, sorted and unique, does not depend on
      // their number.
      const int nth = host_threads(n);
      std::vector<std::vector<uint64_t>> part(nth);
      run_chunks(n, nth, [&](int t, int64_t lo, int64_t hi) {
        std::vector<uint64_t>& out = part[t];
        for (int64_t i = lo; i < hi; ++i) {
          if (!(std::fabs(inc[i]) > threshold(level[i]))) continue;
          for (int p : xs) {
            if (level[i] >> p & 1) continue;
            const uint64_t child = level[i] | ((uint64_t)1 << p);
            if (!structural(child)) out.push_back(child);
          }
        }
        std::sort(out.begin(), out.end());
        out.erase(std::unique(out.begin(), out.end()), out.end());
      });
      std::vector<uint64_t> next = merge_unique(part);
      std::vector<char> keep(next.size());
      run_chunks((int64_t)next.size(), host_threads((int64_t)next.size()),
                 [&](int, int64_t lo, int64_t hi) {
                   for (int64_t i = lo; i < hi; ++i) {
                     const uint64_t child = next[i];
                     int computed = 0;
                     for (uint64_t x = child; x && computed < 2; x &= x - 1) {
                       const uint64_t sub = child & ~(x & (~x + 1));
                       if (std::binary_search(level.begin(), level.end(), sub)) ++computed;
                     }
                     keep[i] = computed >= 2;
                   }
                 });
      size_t kept = 0;
      for (size_t i = 0; i < next.size(); ++i)
        if (keep[i]) next[kept++] = next[i];
      next.resize(kept);
      level.swap(next);
      ++k;
    }
    launch_mbe_total(d_eref, d_eord, K, d_tot, c->stream);
    double tt[2];
    std::vector<double> eo(std::max(K, 1));
    HIPCHK(hipMemcpyAsync(tt, d_tot, 16, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(eo.data(), d_eord, eo.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    *e_ref = tt[0];
    *e_total = tt[1];
    for (int i = 0; i < K; ++i) e_order[i] = eo[i];
    tot.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                             t_start).count();
    tot.ms_tune = c->ms_tune;
    if (stats) *stats = tot;
    sc.done();
  });
}

int64_t mbefci_screened_tuples(mbefci_ctx* c, int32_t order, int32_t* tuples,
                               double* increments) {
  if (!c) return MBEFCI_EINVAL;
  if (order < 1 || order >= (int32_t)c->scr_masks.size()) {
    c->err = "order out of range of the last screened expansion";
    return MBEFCI_EINVAL;
  }
  const auto& ms = c->scr_masks[order];
  const auto& inc = c->scr_inc[order];
  // lexicographic order of the sorted orbital lists
  std::vector<std::vector<int32_t>> lists(ms.size());
  for (size_t i = 0; i < ms.size(); ++i)
    for (uint64_t x = ms[i]; x; x &= x - 1) lists[i].push_back(__builtin_ctzll(x));
  std::vector<size_t> perm(ms.size());
  for (size_t i = 0; i < perm.size(); ++i) perm[i] = i;
  std::sort(perm.begin(), perm.end(), [&](size_t a, size_t b) { return lists[a] < lists[b]; });
  for (size_t r = 0; r < perm.size(); ++r) {
    if (tuples)
      std::copy(lists[perm[r]].begin(), lists[perm[r]].end(), tuples + (int64_t)r * order);
    if (increments) increments[r] = inc[perm[r]];
  }
  return (int64_t)ms.size();
}

int mbefci_mbe_backward(mbefci_ctx* c, const double* grad_out, double* d_h1, double* d_eri,
                        void* stream) {
  return guarded(c, [&] {
    if (!c->plan || !c->plan->is_mbe || !c->have_forward)
      throw Error(MBEFCI_EINVAL, "mbefci_mbe_backward needs a preceding mbefci_mbe_forward on ctx");
    if (!c->opts.keep_ci) throw Error(MBEFCI_EINVAL, "CI vectors were not kept (keep_ci = 0)");
    if (!grad_out || !d_h1 || !d_eri) throw Error(MBEFCI_EINVAL, "null argument");
    Plan& P = *c->plan;
    for (int n = 0; n <= P.max_order; ++n)
      if (!std::isfinite(grad_out[n])) throw Error(MBEFCI_EINVAL, "grad_out holds a non-finite value");
    StreamScope sc(c, stream);
    RdmOut R = rdm_pass(c, P);
    double* d_g = arena<double>(c, "grad_out", P.max_order + 1);
    double* d_w = arena<double>(c, "weights", P.nitem);
    std::vector<double> g(grad_out, grad_out + P.max_order + 1);
    upload(c, d_g, g);
    launch_mbe_weights(P.d_buckets, (int)P.buckets.size(), P.nitem, (int)P.xsorted.size(),
                       P.max_order, d_g, d_w, c->stream);
    uint64_t occmask = 0;
    for (int i = 0; i < P.sp.nO; ++i) occmask |= (uint64_t)1 << P.sp.O[i];
    const int M = P.norb, npair = M * (M - 1) / 2;
    uint64_t* d_live = arena<uint64_t>(c, "grad_live", P.nitem);
    int32_t* d_list = arena<int32_t>(c, "grad_list", (size_t)M * P.nitem);
    int32_t* d_count = arena<int32_t>(c, "grad_count", M);
    int32_t* d_pcount = arena<int32_t>(c, "grad_pcount", std::max(npair, 1));
    int64_t* d_poff = arena<int64_t>(c, "grad_poff", npair + 1);
    launch_grad_index(P.d_items, P.nitem, P.act, occmask, M, d_live, d_list, d_count, d_pcount,
                      d_poff, c->stream);
    HIPCHK(hipGetLastError());
    int64_t nplist = 0;
    HIPCHK(hipMemcpyAsync(&nplist, d_poff + npair, sizeof(int64_t), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    int32_t* d_plist = arena<int32_t>(c, "grad_plist", (size_t)std::max<int64_t>(nplist, 1));
    launch_grad(P.d_items, P.nitem, P.act, occmask, M, d_w, R.rdmp, R.roff, d_live, d_list,
                d_count, d_pcount, d_poff, d_plist, d_h1, d_eri, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    sc.done();
  });
}

int mbefci_probe_peaks(mbefci_ctx* c, double* fp64_mfma_tflops, double* copy_gbps) {
  return guarded(c, [&] {
    if (!fp64_mfma_tflops || !copy_gbps) throw Error(MBEFCI_EINVAL, "null output");
    HIPCHK(hipSetDevice(c->device));
    int ncu = 0;
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
    const int64_t n = (int64_t)32 << 20;  // doubles per copy buffer: 256 MiB
    double* buf = arena<double>(c, "probe", (size_t)(2 * n + 256));
    double* src = buf;
    double* dst = buf + n;
    double* out = buf + 2 * n;
    launch_fill(src, n, 1.0, c->stream);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto timed = [&](auto&& launch, int reps) {
      float best = 1e30f;
      launch();  // warm
      for (int r = 0; r < reps; ++r) {
        HIPCHK(hipEventRecord(e0, c->stream));
        launch();
        HIPCHK(hipEventRecord(e1, c->stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        best = std::min(best, ms);
      }
      return (double)best;
    };
    // sixteen blocks per CU in flight or queued, eight chains per wave: the
    // rate no longer rises with either (measured), about 10 ms per launch
    const int mblocks = 16 * ncu, iters = 2000;
    const double tm = timed([&] { launch_probe_mfma(out, mblocks, iters, c->stream); }, 3);
    const double tc = timed([&] { launch_probe_copy(src, dst, n, 4 * ncu * 8, c->stream); }, 5);
    HIPCHK(hipEventDestroy(e0));
    HIPCHK(hipEventDestroy(e1));
    *fp64_mfma_tflops = probe_mfma_flops(mblocks, iters) / (tm * 1e-3) / 1e12;
    *copy_gbps = 2.0 * n * 8 / (tc * 1e-3) / 1e9;
  });
}

int mbefci_time_kernels(mbefci_ctx* c, int32_t reps, mbefci_kernel_time* out, int32_t cap,
                        int32_t* count) {
  return guarded(c, [&] {
    if (!c->plan || !c->have_forward) throw Error(MBEFCI_EINVAL, "no forward to re-time");
    if (reps < 1 || !count || (cap > 0 && !out)) throw Error(MBEFCI_EINVAL, "invalid arguments");
    HIPCHK(hipSetDevice(c->device));
    Plan& P = *c->plan;
    DavState* backup = arena<DavState>(c, "state_backup", P.nitem);
    HIPCHK(hipMemcpyAsync(backup, P.st, sizeof(DavState) * P.nitem, hipMemcpyDeviceToDevice,
                          c->stream));
    launch_state_unconv(P.d_items, P.st, P.nitem, c->stream);
    // replay whole sigma sweeps exactly as the solver runs them, with events
    // around every launch
    const std::vector<SigmaLaunch> Ls = sigma_launches(P, whole(P));
    std::vector<hipEvent_t> ev(2 * Ls.size());
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    std::vector<double> ms(Ls.size(), 0.0);
    sigma(c, P, whole(P), -1);  // warm
    for (int r = 0; r < reps; ++r) {
      for (size_t k = 0; k < Ls.size(); ++k) {
        HIPCHK(hipEventRecord(ev[2 * k], c->stream));
        sigma_launch(c, P, Ls[k], -1);
        HIPCHK(hipEventRecord(ev[2 * k + 1], c->stream));
      }
      HIPCHK(hipStreamSynchronize(c->stream));
      for (size_t k = 0; k < Ls.size(); ++k) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]));
        ms[k] += t;
      }
    }
    for (auto& e : ev) HIPCHK(hipEventDestroy(e));
    // aggregate per kernel: algorithmic work from the items each launch covers
    std::map<std::string, mbefci_kernel_time> agg;
    std::vector<std::string> order;
    for (size_t k = 0; k < Ls.size(); ++k) {
      const SigmaLaunch& L = Ls[k];
      double nd = 0.0, flops = 0.0, bytes = 0.0;
      std::string name;
      if (L.kind == 0) {
        const Group& g = P.groups[L.group];
        for (int w = L.lo; w < L.lo + L.cnt; ++w)
          if (g.tiles[w].begin == 0) nd += (double)P.items[g.tiles[w].item].ndet;
        const double np = g.n * (g.n + 1) / 2;
        flops = 2.0 * np * np * nd;
        // c read once, G written once (up to kFoldMax orbitals its off-diagonal
        // rows, and sigma's diagonal part)
        bytes = 8.0 * (g.n <= kFoldMax ? 2.0 + np - g.n : 1.0 + np) * nd;
        name = (g.tn < 0 ? "sigma_dgemm_flat<n=" : "sigma_dgemm<n=") + std::to_string(g.n) +
               ",tile=" + std::to_string(g.tn < 0 ? -g.tn : g.tn) + ">";
      } else if (L.kind == 1) {
        for (int w = L.lo; w < L.lo + L.cnt; ++w)
          if (P.segs[w].begin == 0) {
            const Item& I = P.items[P.segs[w].item];
            nd += (double)I.ndet;
            // G read once, sigma written (up to kFoldMax orbitals: G's
            // off-diagonal rows, sigma read and written)
            bytes += 8.0 * (I.n <= kFoldMax ? I.npair - I.n + 2.0 : I.npair + 1.0) * I.ndet;
          }
        name = "sigma_gather";
      } else if (L.kind == 2) {
        // per work unit: its tiles' determinants of the class's irrep space
        const auto& sg = P.sym_groups[L.group];
        for (int w = L.lo; w < L.lo + L.cnt; ++w) {
          const Work& wk = sg.tiles[w];
          const SymInfo& Y = P.item_symtab[wk.item]->host;
          const int cls = wk.pad_ >> 3, ap = wk.pad_ & 7;
          const double nps = Y.cls0[cls + 1] - Y.cls0[cls];
          const int NA = Y.nac[ap], NB = Y.nbc[ap ^ Y.wfn ^ cls];
          const int TN = sym_tile(sg.npc);
          const int bk = wk.begin / NA;
          const double cols = std::min(TN, NB - bk * TN);
          const double d = (wk.end - wk.begin) * cols;
          nd += d;
          flops += 2.0 * nps * nps * d;
          bytes += 8.0 * (1.0 + nps) * d;
        }
        name = "sigma_sym_dgemm<npc=" + std::to_string(sg.npc) + ">";
      } else {
        for (int w = L.lo; w < L.lo + L.cnt; ++w)
          if (P.sym_blocks[w].begin == 0) {
            const Item& I = P.items[P.sym_blocks[w].item];
            const SymInfo& Y = P.item_symtab[P.sym_blocks[w].item]->host;
            nd += (double)I.ndet;
            bytes += 8.0 * ((double)Y.gsize + I.ndet);  // G read once, sigma written once
          }
        name = "sigma_sym_gather";
      }
      if (!agg.count(name)) {
        order.push_back(name);
        mbefci_kernel_time z{};
        std::snprintf(z.name, sizeof(z.name), "%s", name.c_str());
        agg[name] = z;
      }
      mbefci_kernel_time& a = agg[name];
      a.launches += 1;
      a.ms_per_launch += ms[k] / reps;
      a.flops += flops;
      a.bytes += bytes;
      a.ndet += nd;
    }
    std::vector<mbefci_kernel_time> recs;
    for (const std::string& nm : order) {
      mbefci_kernel_time a = agg[nm];
      a.ms_per_launch /= a.launches;
      a.flops /= a.launches;
      a.bytes /= a.launches;
      a.ndet /= a.launches;
      recs.push_back(a);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(P.st, backup, sizeof(DavState) * P.nitem, hipMemcpyDeviceToDevice,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int n = std::min<int>((int)recs.size(), cap);
    for (int i = 0; i < n; ++i) out[i] = recs[i];
    *count = (int32_t)recs.size();
  });
}

}  // extern "C"
