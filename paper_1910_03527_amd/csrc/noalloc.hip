// sigma = H c of one CASCI without any device allocation, for callers that
// cannot allocate (code under HIP graph capture, tight serving loops).
//
// Every intermediate of the sigma build (string, link and pair tables, the
// folded Hamiltonian record, the pair-space matrix W, the contracted pair
// array G, work lists) lives in one file-scope device array, `scratch`, of
// kScratchBytes per GPU, held until the process ends.  Host code never passes
// the array's name to a kernel: its device address is taken once per device
// with hipGetSymbolAddress (noalloc_init, called when a context is created,
// or on the first call on a device) and kept in g_scratch[device].  The
// kernels are those of mbefci_sigma (kernels.hip); only the storage differs.
// Calls that overlap on one GPU share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "common.h"
#include "launch.h"
#include "mbefci.h"

namespace mbefci {

constexpr size_t kScratchBytes = (size_t)32 << 20;  // 32 MiB per GPU
constexpr int kNoallocMaxDevices = 64;
constexpr int kNoallocTile = 32;  // one alpha string x 32 beta strings per tile
constexpr int kNoallocTpw = 16;   // tiles per workgroup

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mutex;
void* g_scratch[kNoallocMaxDevices] = {};

int64_t binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Byte offsets of every array in the scratch, each on a 256-byte boundary.
struct Layout {
  size_t item, ham, st, hptr, gptr, ecore, tiles, segs, block, diag;
  size_t strA, strB, linkA, linkAT, linkB, linkBT, pairA, pairAT, pairB, pairBT, W, G;
  size_t total;
  int ntiles, nsegs;
};

Layout layout(int n, int64_t Na, int64_t Nb, int La, int Lb) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) & ~(size_t)255;
    return at;
  };
  const int64_t npair = (int64_t)n * (n + 1) / 2;
  const int64_t kpad = (npair + 15) / 16 * 16;
  const int64_t nblk = (Nb + kNoallocTile - 1) / kNoallocTile;
  L.ntiles = (int)(nblk * ((Na + kNoallocTpw - 1) / kNoallocTpw));
  const int64_t nsg = Na * ((Nb + 63) / 64);
  L.nsegs = (int)((nsg + 3) / 4);
  L.item = take(sizeof(Item));
  L.ham = take(sizeof(ItemHam));
  L.st = take(sizeof(DavState));
  L.hptr = take(sizeof(double*));
  L.gptr = take(sizeof(double*));
  L.ecore = take(sizeof(double));
  L.tiles = take(sizeof(Work) * (size_t)L.ntiles);
  L.segs = take(sizeof(Work) * (size_t)L.nsegs);
  L.block = take(sizeof(Work));
  L.diag = take(sizeof(double));
  L.strA = take(sizeof(uint64_t) * Na);
  L.strB = take(sizeof(uint64_t) * Nb);
  L.linkA = take(sizeof(uint32_t) * Na * La);
  L.linkAT = take(sizeof(uint32_t) * Na * La);
  L.linkB = take(sizeof(uint32_t) * Nb * Lb);
  L.linkBT = take(sizeof(uint32_t) * Nb * Lb);
  L.pairA = take(sizeof(int32_t) * Na * npair);
  L.pairAT = take(sizeof(int32_t) * Na * npair);
  L.pairB = take(sizeof(int32_t) * Nb * npair);
  L.pairBT = take(sizeof(int32_t) * Nb * npair);
  L.W = take(sizeof(double) * kpad * kpad);
  L.G = take(sizeof(double) * npair * Na * g_stride((int)Nb));
  L.total = off;
  return L;
}

// Writes the CASCI record, the integral pointers, the solver state of a single
// caller vector in slot 0 and the work lists of the contraction (tiles of
// kNoallocTile columns, kNoallocTpw alpha strings per unit, never crossing a
// beta block), the gather (four row-aligned 64-determinant segments per unit)
// and the diagonal (one 256-determinant block).  One block of 256 threads.
__global__ void k_noalloc_prepare(Item item, Item* items, const double* h1, const double* eri,
                                  double e_core, const double** hptr, const double** gptr,
                                  double* ecore, DavState* st, Work* tiles, int ntiles,
                                  Work* segs, int nsegs, Work* block) {
  const int t = threadIdx.x;
  if (t == 0) {
    items[0] = item;
    hptr[0] = h1;
    gptr[0] = eri;
    ecore[0] = e_core;
    DavState s{};
    s.m = 1;
    s.nguess = 1;
    st[0] = s;
    block[0] = Work{0, 0, 1, 0};
  }
  const int Na = item.Na, Nb = item.Nb;
  const int per_blk = (Na + kNoallocTpw - 1) / kNoallocTpw;
  for (int w = t; w < ntiles; w += blockDim.x) {
    const int bk = w / per_blk, a = (w % per_blk) * kNoallocTpw;
    const int hi = a + kNoallocTpw < Na ? a + kNoallocTpw : Na;
    tiles[w] = Work{0, bk * Na + a, bk * Na + hi, 0};
  }
  const int nsg = Na * ((Nb + 63) / 64);
  for (int w = t; w < nsegs; w += blockDim.x) segs[w] = Work{0, w, nsg, 0};
}

}  // namespace

// The scratch address on `device` (which must be current).  Returns
// hipSuccess, or the error of hipGetSymbolAddress.
hipError_t noalloc_init(int device) {
  if (device < 0 || device >= kNoallocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (g_scratch[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[device] = p;
  return hipSuccess;
}

// sigma = H c (e_core included) of the CASCI (n, na, nb) with active-space
// integrals h1 [n*n] and eri [n^4] (device), c and sigma device [Na*Nb], on
// stream s of `device` (current).  Returns MBEFCI_OK, or an error code with
// *why set; validates sizes only (the integrals are not read on the host).
int noalloc_sigma(int device, int n, int na, int nb, const double* h1, const double* eri,
                  double e_core, const double* c, double* sigma, hipStream_t s, std::string* why) {
  if (n < 0 || n > 14 || na < 0 || nb < 0 || na > n || nb > n) {
    *why = "invalid CASCI shape (norb 0..14, 0 <= nalpha, nbeta <= norb)";
    return MBEFCI_EINVAL;
  }
  if (!h1 || !eri || !c || !sigma) {
    *why = "null pointer";
    return MBEFCI_EINVAL;
  }
  const int64_t Na = binom(n, na), Nb = binom(n, nb);
  const int La = na * (n - na + 1), Lb = nb * (n - nb + 1);
  const Layout L = layout(n, Na, Nb, La, Lb);
  if (L.total > kScratchBytes) {
    *why = "CASCI (" + std::to_string(n) + "," + std::to_string(na) + "," + std::to_string(nb) +
           ") needs " + std::to_string(L.total) + " bytes of scratch; the no-allocation sigma holds " +
           std::to_string(kScratchBytes) + " bytes (32 MiB) per GPU";
    return MBEFCI_ENOMEM;
  }
  hipError_t e = noalloc_init(device);
  if (e != hipSuccess) {
    *why = std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e);
    return MBEFCI_EDEVICE;
  }
  unsigned char* base = (unsigned char*)g_scratch[device];
  auto at = [&](size_t off) { return (void*)(base + off); };
  Item I{};
  I.n = n;
  I.na = na;
  I.nb = nb;
  I.npair = n * (n + 1) / 2;
  I.Na = (int32_t)Na;
  I.Nb = (int32_t)Nb;
  I.La = La;
  I.Lb = Lb;
  I.ndet = Na * Nb;
  I.off = 0;
  I.goff = 0;
  I.woff = 0;
  I.kpad = (I.npair + 15) / 16 * 16;
  I.ham = 0;
  I.chunk0 = 0;
  I.nchunk = 0;
  I.shape = 0;
  I.linkA = (const uint32_t*)at(L.linkA);
  I.linkB = (const uint32_t*)at(L.linkB);
  I.linkBT = (const uint32_t*)at(L.linkBT);
  I.strA = (const uint64_t*)at(L.strA);
  I.strB = (const uint64_t*)at(L.strB);
  I.pairA = (const int32_t*)at(L.pairA);
  I.pairB = (const int32_t*)at(L.pairBT);
  Item* items = (Item*)at(L.item);
  ItemHam* hams = (ItemHam*)at(L.ham);
  DavState* st = (DavState*)at(L.st);
  const double** hptr = (const double**)at(L.hptr);
  const double** gptr = (const double**)at(L.gptr);
  double* ecore = (double*)at(L.ecore);
  Work* tiles = (Work*)at(L.tiles);
  Work* segs = (Work*)at(L.segs);
  Work* block = (Work*)at(L.block);
  double* W = (double*)at(L.W);
  double* G = (double*)at(L.G);
  hipLaunchKernelGGL(k_noalloc_prepare, dim3(1), dim3(256), 0, s, I, items, h1, eri, e_core,
                     hptr, gptr, ecore, st, tiles, L.ntiles, segs, L.nsegs, block);
  launch_strings(n, na, Na, (uint64_t*)at(L.strA), s);
  launch_strings(n, nb, Nb, (uint64_t*)at(L.strB), s);
  launch_links(n, na, Na, (uint32_t*)at(L.linkA), (uint32_t*)at(L.linkAT), nullptr, s);
  launch_links(n, nb, Nb, (uint32_t*)at(L.linkB), (uint32_t*)at(L.linkBT), nullptr, s);
  launch_pair_table(n, na, Na, (int32_t*)at(L.pairA), (int32_t*)at(L.pairAT), s);
  launch_pair_table(n, nb, Nb, (int32_t*)at(L.pairB), (int32_t*)at(L.pairBT), s);
  launch_casci_setup(n, hptr, gptr, ecore, items, 1, hams, W, s);
  if (I.ndet > 1) {
    // the caller's vectors stand in for slot 0 of the solver arenas
    if (!launch_sigma_dgemm(n, kNoallocTile, items, tiles, L.ntiles, W, c, I.ndet, G, sigma, st,
                            0, s)) {
      *why = "no sigma kernel for n=" + std::to_string(n);
      return MBEFCI_EUNSUPPORTED;
    }
    launch_sigma_gather(items, segs, L.nsegs, G, sigma, I.ndet, st, 0,
                        gather_lds_bytes((int64_t)I.npair * g_stride(I.Nb) * 8), s);
    launch_axpy_out(sigma, sigma, c, e_core, I.ndet, s);
  } else {
    double* diag = (double*)at(L.diag);
    launch_hdiag(items, block, 1, hams, diag, s);
    launch_diag_times(sigma, diag, c, e_core, 1, s);
  }
  e = hipGetLastError();
  if (e != hipSuccess) {
    *why = std::string("kernel launch: ") + hipGetErrorString(e);
    return MBEFCI_EDEVICE;
  }
  return MBEFCI_OK;
}

}  // namespace mbefci
