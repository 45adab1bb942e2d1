// Kernel launchers (kernels.hip) called by the host runtime (runtime.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace mbefci {

void launch_strings(int n, int ne, int64_t N, uint64_t* out, hipStream_t s);
void launch_links(int n, int ne, int64_t N, uint32_t* packed, uint32_t* packedT, int32_t* abi4,
                  hipStream_t s);
void launch_pair_table(int n, int ne, int64_t N, int32_t* out, int32_t* outT, hipStream_t s);
void launch_mbe_setup(const MbeSpaces* sp, const BucketDev* buckets, int nbucket, const Item* items,
                      int nitem, const double* h1, const double* eri, double e_const,
                      ItemHam* hams, double* warena, int32_t* tuple_pos, int max_order,
                      int32_t* act_out, hipStream_t s);
void launch_casci_setup(int n, const double* const* h1s, const double* const* eris,
                        const double* ecores, const Item* items, int nitem, ItemHam* hams,
                        double* warena, hipStream_t s);
void launch_hdiag(const Item* items, const Work* work, int nwork, const ItemHam* hams,
                  double* diag, hipStream_t s);
// tn: 32, 64 or 128 columns of one alpha string per tile; -32 or -64: flattened
// tiles of that many consecutive determinants (active spaces of at most 9).
// Up to kFoldMax orbitals it also writes the diagonal pairs' part of sigma to
// Sv (the slot of the vector it reads from V), to which launch_sigma_gather
// then adds the off-diagonal links.
bool launch_sigma_dgemm(int n, int tn, const Item* items, const Work* work, int nwork,
                        const double* warena, const double* V, int64_t ntot, double* G,
                        double* Sv, const DavState* st, int slot, hipStream_t s);
// lds: bytes of LDS reserved per workgroup (the kernel uses none), a cap on
// the workgroups per CU: see gather_lds_bytes
void launch_sigma_gather(const Item* items, const Work* work, int nwork, const double* G,
                         double* Sv, int64_t ntot, const DavState* st, int slot, int lds,
                         hipStream_t s);
// The gather's LDS reservation for items whose row block of G (npair rows
// of the row stride) takes `row_block` bytes.  Each workgroup reads one
// row block scattered; with many resident workgroups the L2 re-fetches it.
// Measured (eight workgroups per CU uncapped): blocks of 112 KB (10
// orbitals) do best at six per CU, blocks of 1 MB and more (13-14
// orbitals) at four; blocks below 64 KB (9 orbitals and fewer) are not
// capped.  (Sized by all npair rows; up to 10 orbitals G holds npair - n.)
inline int gather_lds_bytes(int64_t row_block) {
  if (row_block >= ((int64_t)1 << 20)) return 40960;  // four workgroups per CU
  if (row_block >= 64 * 1024) return 26624;           // six
  return 0;
}
// point-group blocked sigma (items with a SymInfo): the per-class contraction
// (npc = the class's pair count rounded up to 16, sym_npc; work units carry
// class and alpha irrep in Work.pad_ = s * 8 + a') and the gather (work units
// of 256 consecutive determinants)
int sym_npc(int npair_class);
int sym_tile(int npc);  // beta strings per tile of the class's contraction
bool launch_sigma_sym_dgemm(int npc, const Item* items, const Work* work, int nwork,
                            const double* warena, const double* V, int64_t ntot, double* G,
                            const DavState* st, int slot, hipStream_t s);
void launch_sigma_sym_gather(const Item* items, const Work* work, int nwork, const double* G,
                             double* Sv, int64_t ntot, const DavState* st, int slot,
                             hipStream_t s);
// finiteness and 8-fold symmetry of h1 [M*M], eri [M^4]: bits of *flags
// (which must be zero beforehand) as documented at the kernel
void launch_check_integrals(const double* h1, const double* eri, int M, int* flags,
                            hipStream_t s);
void launch_fill(double* p, int64_t n, double v, hipStream_t s);
// peak probes: FP64 MFMA chains (256-thread blocks; flops of one launch from
// probe_mfma_flops) and a copy of n doubles (n even, 16-byte aligned)
void launch_probe_mfma(double* out, int blocks, int iters, hipStream_t s);
double probe_mfma_flops(int blocks, int iters);
void launch_probe_copy(const double* src, double* dst, int64_t n, int blocks, hipStream_t s);
void launch_dav_guess(const Item* items, int ibase, int nitem, const double* diag, double* V,
                      int64_t ntot, DavState* st, int nguess, hipStream_t s);
void launch_dav_dots(const Item* items, const Work* chunks, int nchunk, const double* V,
                     const double* Sv, int64_t ntot, const DavState* st, int slot, double* part,
                     hipStream_t s);
void launch_dav_rr(const Item* items, int ibase, int nitem, const double* part, DavState* st,
                   int slot, hipStream_t s);
// P-space arrays of a plan: pidx [item][kMaxPspace] determinant addresses,
// pQ [item][kMaxPspace^2] orthogonal factor of H_PP = Q T Q^T (row = P
// position), pT [item][2][kMaxPspace] diagonal and off-diagonal of T, pdots
// [item][kMaxSpace] Gram-Schmidt dot corrections.
struct PspaceArgs {
  const int32_t* pidx;
  const double* pQ;
  const double* pT;
  double* pdots;
};
// chunked P-space selection of large CASCIs: per chunk of kSelectChunk
// determinants a work unit (item, chunk, first candidate slot of the item),
// per item its first slot or -1, and the candidate keys (kMaxPspace per slot)
constexpr int64_t kSelectChunk = 16384;
// Row stride of G (doubles): the beta-string count rounded up to 16, so
// that every row of G starts on a 128-byte line, when that adds at most
// 1/16 to the row (252 -> 256, 3432 -> 3440); short rows, where padding
// would grow G by up to 60%, keep their length.  Item offsets into G are
// multiples of 16 doubles.
__host__ __device__ inline int g_stride(int nb) {
  const int p = (nb + 15) & ~15;
  return (p - nb) * 16 <= nb ? p : nb;
}
// P-space size of a CASCI of nd determinants: its whole space up to
// kMaxPspace determinants, else min(pmax, nd / kPspaceRatio) when that
// reaches kPspaceMinDim, else 0 (unit-vector guess, diagonal correction).
constexpr int kPspaceRatio = 64;
constexpr int kPspaceMinDim = 24;
__host__ __device__ inline int pspace_dim(int64_t nd, int pmax) {
  if (nd <= kMaxPspace) return (int)nd;
  const int64_t p = nd / kPspaceRatio < pmax ? nd / kPspaceRatio : pmax;
  return p >= kPspaceMinDim ? (int)p : 0;
}
// Which P-space reduction a CASCI takes: a P-space of a larger CASCI of
// 0 more than kPspaceMid, 4 at most kPspaceMid determinants; its whole space
// of 1 at most kExactSmall, 2 at most kExactMid, 3 at most kMaxPspace
// determinants; -1 none (a single determinant or unit-vector guesses).
constexpr int kExactSmall = 36;
constexpr int kExactMid = 100;
constexpr int kPspaceMid = 76;
constexpr int kPspaceClasses = 5;
__host__ __device__ inline int pspace_class(int64_t nd, int pmax) {
  const int p = nd <= 1 ? 0 : pspace_dim(nd, pmax);
  if (p == 0) return -1;
  if (nd > kMaxPspace) return p <= kPspaceMid ? 4 : 0;
  return nd <= kExactSmall ? 1 : nd <= kExactMid ? 2 : 3;
}
// per class, the items of a view that take it (absolute indices, ascending)
struct PspaceLists {
  const int32_t* list[kPspaceClasses];
  int n[kPspaceClasses];
};
struct PspaceSelect {
  const Work* work;
  int nwork;
  const int32_t* slot;
  uint64_t* hi;
  uint32_t* lo;
};
void launch_pspace_setup(const Item* items, int ibase, int nitem, const PspaceLists& pl,
                         const ItemHam* hams, const double* diag, int32_t* pidx, double* pQ,
                         double* pT, double* V, int64_t ntot, DavState* st, int pmax, int nunit,
                         const PspaceSelect& sel, hipStream_t s);
// One Davidson iteration after a sigma sweep: restart, correction, Gram-Schmidt.
// olsen_all: every item takes the Olsen correction (Rb, Xb: residual and Ritz
// vector buffers); otherwise the diagonal correction (with the P-space block
// when ps is set), and items whose residual fell below olsen_below (> 0)
// switch to the Olsen correction for the rest of the solve.
void launch_dav_iteration(const Item* items, int ibase, int nitem, const Work* chunks, int nchunk,
                          double* V, double* Sv, const double* diag, int64_t ntot, DavState* st,
                          double* part, double tol, int max_iter, int mmax, double* Rb,
                          double* Xb, const PspaceArgs* ps, bool olsen_all, double olsen_below,
                          hipStream_t s);
void launch_item_energy(const Item* items, const ItemHam* hams, const DavState* st, int nitem,
                        double* f, hipStream_t s);
void launch_mbe_combine(const MbeSpaces* sp, const BucketDev* buckets, int nbucket,
                        const int32_t* tuple_pos, int max_order, const double* f, int nitem,
                        double* inc, double* inc_lex, double* f_lex, const int64_t* order_off,
                        const int32_t* xpos_o, const int32_t* xpos_v, int nX, double* e_order,
                        hipStream_t s);

void launch_count_active(const DavState* st, int ibase, int nitem, int* out, hipStream_t s);
void launch_collect(const DavState* st, int nitem, int32_t* out, hipStream_t s);
void launch_state_single(DavState* st, hipStream_t s);
void launch_axpy_out(double* out, const double* sv, const double* c, double a, int64_t n,
                     hipStream_t s);
void launch_diag_times(double* out, const double* d, const double* c, double a, int64_t n,
                       hipStream_t s);
void launch_add_scalar(double* out, const double* in, double a, int64_t n, hipStream_t s);
void launch_ritz_vector(const Item* items, const Work* chunks, int nchunk, const double* V,
                        int64_t ntot, const DavState* st, double* out, hipStream_t s);
void launch_state_unconv(const Item* items, DavState* st, int nitem, hipStream_t s);
void launch_mbe_total(const double* f, const double* e_order, int k, double* out, hipStream_t s);

bool launch_rdm_syrk(int n, int tn, const Item* items, const Work* work, int nwork,
                     const double* civ, double* part, hipStream_t s);
void launch_rdm_reduce(const Item* items, int nitem, const int32_t* wlo, const int32_t* whi,
                       const double* part, const int64_t* poff, double* rdmp, const int64_t* roff,
                       hipStream_t s);
void launch_mbe_weights(const BucketDev* buckets, int nbucket, int nitem, int nexp, int max_order,
                        const double* g, double* w, hipStream_t s);
// dE/dh and dE/d(pq|rs) from the weighted RDMs, in two launches around a
// host read of poff[M (M - 1) / 2] (the length of the pair lists).
// launch_grad_index fills the workspace: live [nitem] masks, per-orbital
// item lists list [M * nitem] and count [M], pair counts pcount
// [M (M - 1) / 2] and offsets poff [M (M - 1) / 2 + 1]; launch_grad fills
// the pair lists plist [poff[M (M - 1) / 2]] and sums the gradients.
void launch_grad_index(const Item* items, int nitem, const int32_t* act, uint64_t occmask, int M,
                       uint64_t* live, int32_t* list, int32_t* count, int32_t* pcount,
                       int64_t* poff, hipStream_t s);
void launch_grad(const Item* items, int nitem, const int32_t* act, uint64_t occmask, int M,
                 const double* w, const double* rdmp, const int64_t* roff, const uint64_t* live,
                 const int32_t* list, const int32_t* count, const int32_t* pcount,
                 const int64_t* poff, int32_t* plist, double* dh, double* dg, hipStream_t s);
void launch_casci_rdm_out(const Item* items, int it, int n, const double* rdmp,
                          const int64_t* roff, double* rdm1, double* rdm2, hipStream_t s);

constexpr int kChunkElems = 4096;   // elements per Davidson reduction chunk
constexpr int kPartStride = kMaxSpace + 2;

// screened expansion: the computed tuples of every order (masks ascending)
struct ScreenArrays {
  const uint64_t* mask[kMaxActive + 1];
  const double* inc[kMaxActive + 1];
  int64_t n[kMaxActive + 1];
};
void launch_mbe_setup_list(const MbeSpaces* sp, const uint64_t* masks, const Item* items, int nitem,
                           const double* h1, const double* eri, double e_const, ItemHam* hams,
                           double* warena, hipStream_t s);
void launch_screen_increments(const uint64_t* masks, int64_t n, int k, const double* f,
                              const double* e_ref, const ScreenArrays& lower, double* inc,
                              double* order_sum, hipStream_t s);
}  // namespace mbefci

