// Shared internal definitions of the MBE-FCI HIP library (gfx950, FP64).
//
// Notation follows the paper (arXiv:1910.03527): M molecular orbitals, a
// reference space R and an expansion space X; every tuple T of expansion
// orbitals defines one CASCI in the active set A = R u T (Eq. 1, Eq. 2).
// Inside one CASCI: n active orbitals, na/nb active alpha/beta electrons,
// Na = C(n,na) alpha strings, Nb = C(n,nb) beta strings, determinant
// address K = Ka*Nb + Kb, npair = n(n+1)/2 orbital pairs (a >= b).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbefci {

constexpr int kMaxActive = 16;          // active orbitals per CASCI
constexpr int kMaxPair = kMaxActive * (kMaxActive + 1) / 2;
constexpr int kMaxOrb = 64;             // orbitals of the whole problem
constexpr int kMaxSpace = 16;           // Davidson subspace (+1 correction slot)
constexpr int kBinom = 65;              // binomial table C(n,k), n,k < 65
constexpr int kMaxPspace = 112;         // P-space (lowest-diagonal determinants) size cap

// packed single-excitation link: bits 0..21 string address J, bits 22..29
// orbital-pair index pair(p,q) = max(p,q)*(max(p,q)+1)/2 + min(p,q),
// bit 31 set when the sign is negative.
__host__ __device__ inline uint32_t pack_link(int J, int pair, int sign) {
  return (uint32_t)J | ((uint32_t)pair << 22) | (sign < 0 ? 0x80000000u : 0u);
}
__host__ __device__ inline int link_addr(uint32_t e) { return (int)(e & 0x3FFFFFu); }
__host__ __device__ inline int link_pair(uint32_t e) { return (int)((e >> 22) & 0xFFu); }
__host__ __device__ inline double link_sign(uint32_t e) { return (e & 0x80000000u) ? -1.0 : 1.0; }
__host__ __device__ inline int pair_index(int p, int q) {
  int a = p > q ? p : q, b = p > q ? q : p;
  return a * (a + 1) / 2 + b;
}
// index of the off-diagonal pair a > b among the n (n - 1) / 2 such pairs
__host__ __device__ inline int offdiag_index(int a, int b) { return a * (a - 1) / 2 + b; }
// Active spaces of up to kFoldMax orbitals: the sigma contraction sums the
// diagonal pairs' part of sigma itself and G holds only the off-diagonal pair
// rows; larger ones keep every pair row in G (their contraction kernels have
// no register room for the epilogue).
constexpr int kFoldMax = 10;

// Load through the global address space (pointers read from device structs
// are generic; this keeps the loads off the flat path).
template <class T>
__device__ inline T ldg(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}

// Load through the constant address space: lets the compiler use scalar
// loads when the address is wave-uniform (read-only tables).
template <class T>
__device__ inline T ldc(const T* p) {
  return *(const __attribute__((address_space(4))) T*)p;
}

// Point-group blocking (abelian groups: D2h and its subgroups).  Irreps are
// labels 0..7 whose product is their XOR; a string's irrep is the XOR of its
// occupied orbitals' labels.  The strings of each spin are sorted by (irrep,
// bitmask), and the CI vector of irrep G holds only the determinants of that
// irrep: blocks over the alpha irreps a = 0..7, block a = [nac[a]][nbc[a^G]]
// (alpha strings of irrep a times beta strings of irrep a^G) at offset
// blk[a].  A one-body operator E_pq changes the irrep by the pair class
// s = irr(p)^irr(q), and the pair-space matrix W couples only pairs of one
// class, so sigma splits into one contraction per class s on the
// determinants of irrep G^s: G_s = W_s D+_s.  Pairs are listed class by class
// (positions cls0[s] .. cls0[s+1]-1), and G_s is stored per alpha irrep a' of
// the irrep-G^s space as [nac[a']][npair_s][nbc[a'^G^s]] at gofs[s][a'].
constexpr int kIrreps = 8;
struct SymInfo {
  int32_t wfn;                       // irrep G of the solved state
  int32_t npair;                     // pairs in all classes (n(n+1)/2)
  int32_t na0[kIrreps], nac[kIrreps];  // first sorted alpha string of each irrep, count
  int32_t nb0[kIrreps], nbc[kIrreps];  // the same for beta strings
  int64_t blk[kIrreps + 1];          // CI block offsets (blk[8] = determinants of irrep G)
  int32_t cls0[kIrreps + 1];         // class-sorted pair positions of class s
  int32_t pair_of[kMaxPair];         // class-sorted position -> pair index a(a+1)/2+b
  int8_t cls_of[kMaxPair];           // class-sorted position -> its class
  int64_t gofs[kIrreps][kIrreps];    // G_s block of alpha irrep a', from the item's G
  int64_t gsize;                     // doubles of all G_s blocks
};

// One CASCI problem inside a batch.
struct Item {
  int32_t n, na, nb, npair;
  int32_t Na, Nb, La, Lb;
  int64_t ndet;           // Na*Nb
  int64_t off;            // offset of this item in every vector slot of the arenas
  int64_t goff;           // offset of its G block [npair][ndet]
  int64_t woff;           // offset of its W matrix [kpad][kpad] (row-major)
  int32_t kpad;           // npair rounded up to a multiple of 16
  int32_t ham;            // index of its ItemHam record
  int32_t chunk0, nchunk; // partial-reduction chunks [chunk0, chunk0+nchunk)
  int32_t shape;          // index of its string/link table set
  int32_t pad_;
  const uint32_t* linkA;  // [Na][La]
  const uint32_t* linkB;  // [Nb][Lb]
  const uint32_t* linkBT; // [Lb][Nb] (link-major copy: coalesced per-lane reads)
  const uint64_t* strA;   // [Na] alpha string bitmasks
  const uint64_t* strB;   // [Nb] beta string bitmasks
  const int32_t* pairA;   // [Na][npair] pair table (see pack_pair_entry)
  const int32_t* pairB;   // [npair][Nb] the same for beta strings, pair-major
  // point-group blocked CASCI (null: the plain [Na][Nb] layout).  Then strA,
  // strB are sorted by (irrep, bitmask); links and pair tables hold string
  // indices local to their irrep and class-sorted pair positions; linkA
  // [Na][La], linkB [Nb][Lb], pairA [Na][npair], pairB [npair][Nb]; ndet is
  // the number of determinants of irrep sym->wfn.
  const SymInfo* sym;
};

// The alpha and beta strings of determinant K of item I, in either layout.
__host__ __device__ inline void det_strings(const Item& I, int64_t K, uint64_t& ma,
                                            uint64_t& mb) {
  if (!I.sym) {
    ma = I.strA[K / I.Nb];
    mb = I.strB[K % I.Nb];
    return;
  }
  const SymInfo& S = *I.sym;
  int a = 0;
  while (a < kIrreps - 1 && K >= S.blk[a + 1]) ++a;
  const int b = a ^ S.wfn;
  const int64_t loc = K - S.blk[a];
  ma = I.strA[S.na0[a] + loc / S.nbc[b]];
  mb = I.strB[S.nb0[b] + loc % S.nbc[b]];
}

// Pair table entry of string K and orbital pair (a >= b): the single
// excitation among E_ab K, E_ba K that does not vanish (at most one does for
// a != b; E_aa K = K when a is occupied), stored as ((J + 1) << 1) | neg,
// 0 when both vanish.
__host__ __device__ inline int32_t pack_pair_entry(int J, int sign) {
  return ((J + 1) << 1) | (sign < 0 ? 1 : 0);
}

// Active-space Hamiltonian of one CASCI after the frozen-core fold.
struct ItemHam {
  double ecore;                          // constant + frozen-core energy
  double heff[kMaxActive * kMaxActive];  // h_eff_tu
  double J[kMaxActive * kMaxActive];     // (tt|uu)
  double K[kMaxActive * kMaxActive];     // (tu|ut)
  const double* eri;                     // (pq|rs) of the whole problem, [M^4]
  int32_t M;                             // its orbital count
  int32_t act[kMaxActive];               // active orbital t -> orbital of the problem
};

// Per-item Davidson state (device resident).
struct DavState {
  int32_t m;          // current subspace size
  int32_t conv;       // 1 once converged
  int32_t iters;      // iterations taken
  int32_t status;     // 0 ok, 1 not converged, 2 breakdown
  int32_t nguess;     // number of guess vectors (slots 0..nguess-1)
  int32_t np;         // P-space size (0: diagonal preconditioner only)
  int32_t onepass;    // this iteration's correction needs one Gram-Schmidt pass
  int32_t olsen;      // 1: the corrections have switched to the Olsen form
  double theta;       // lowest Ritz value (active-space energy without ecore)
  double rnorm;       // residual norm of the last Ritz vector
  double tnorm2;      // squared norm of the correction vector
  double eps;         // Olsen shift of the correction equation
  double y[kMaxSpace];
  double yp[kMaxSpace];   // Ritz coefficients of the previous iteration (restart)
  double coef[kMaxSpace + 1];
  double Hs[kMaxSpace * kMaxSpace];
};

// One bucket of MBE tuples: every tuple of a given order with a given number
// of occupied (reference-determinant) orbitals; all share one CASCI shape.
struct BucketDev {
  int32_t order, nocc;
  int64_t item0, count;
};

// The orbital partition of an MBE problem for the device: the expansion space
// split into its occupied part Xo and virtual part Xv (each sorted), the
// reference space R and the occupied set O of the reference determinant.
struct MbeSpaces {
  int M, nocc_ref;  // nocc_ref = |O n R|
  int nR, nXo, nXv, nO;
  int R[kMaxOrb];
  int Xo[kMaxOrb];
  int Xv[kMaxOrb];
  int O[kMaxOrb];
};

struct Work {     // one unit of a segmented launch: an item and a range
  int32_t item;
  int32_t begin;  // first tile / chunk
  int32_t end;    // one past the last
  int32_t pad_;
};

}  // namespace mbefci
