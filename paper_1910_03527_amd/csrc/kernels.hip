// HIP kernels of the MBE-FCI hot path for gfx950 (CDNA4), all FP64.
//
// One translation unit holds every kernel so that the binomial table lives in
// a single __constant__ object.  Launchers at the bottom are the only symbols
// the host runtime calls (declared in launch.h).
#include <type_traits>

#include "common.h"
#include "launch.h"

namespace mbefci {

// ----------------------------------------------------------------- binomials
struct BinomTable {
  int64_t v[kBinom][kBinom];
};
constexpr BinomTable make_binom() {
  BinomTable t{};
  for (int n = 0; n < kBinom; ++n) {
    t.v[n][0] = 1;
    for (int k = 1; k <= n; ++k) t.v[n][k] = t.v[n - 1][k - 1] + (k <= n - 1 ? t.v[n - 1][k] : 0);
  }
  return t;
}
__constant__ BinomTable c_binom = make_binom();

__device__ inline int64_t binom(int n, int k) {
  return (n < 0 || k < 0 || k > n) ? 0 : c_binom.v[n][k];
}

// Address of a string (bitmask, ascending-integer order of all strings with
// the same popcount): combinatorial number system sum_j C(o_j, j), o_j the
// j-th occupied orbital (1-based j) in ascending order.
__device__ inline int64_t string_addr(uint64_t mask) {
  int64_t a = 0;
  int j = 1;
  while (mask) {
    int o = __builtin_ctzll(mask);
    a += binom(o, j++);
    mask &= mask - 1;
  }
  return a;
}

// Inverse of string_addr for strings of ne electrons.
__device__ inline uint64_t string_unrank(int64_t r, int n, int ne) {
  uint64_t mask = 0;
  int o = n - 1;
  for (int j = ne; j >= 1; --j) {
    while (binom(o, j) > r) --o;
    mask |= (uint64_t)1 << o;
    r -= binom(o, j);
    --o;
  }
  return mask;
}

// Lexicographic rank / unrank of a sorted k-combination of {0..N-1}.
__device__ inline int64_t comb_lex_rank(const int* c, int k, int N) {
  int64_t r = 0;
  int prev = -1;
  for (int i = 0; i < k; ++i) {
    for (int j = prev + 1; j < c[i]; ++j) r += binom(N - 1 - j, k - 1 - i);
    prev = c[i];
  }
  return r;
}
__device__ inline void comb_lex_unrank(int64_t r, int k, int N, int* c) {
  int j = 0;
  for (int i = 0; i < k; ++i) {
    while (true) {
      int64_t b = binom(N - 1 - j, k - 1 - i);
      if (r < b) break;
      r -= b;
      ++j;
    }
    c[i] = j++;
  }
}

// ------------------------------------------------- strings and link tables
__global__ void k_strings(int n, int ne, int64_t N, uint64_t* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) out[i] = string_unrank(i, n, ne);
}

// One thread per string I: its single-excitation links E_pq|I> = s|J> in the
// canonical order (diagonal entries first, then q in I ascending, p not in I
// ascending).  The sign is (-1)^(number of occupied orbitals strictly between
// p and q), the parity of a+_p a_q acting on the occupation-number vector.
// abi4 lists (p, q, J, s).  The packed tables are the sigma gather's.  Up
// to kFoldMax orbitals an off-diagonal entry carries G's row
// offdiag_index(max(p, q), min(p, q)) (the diagonal entries, first in packed,
// carry pair_index(o, o) and the gather skips them) and the link-major copy
// packedT holds only the L - ne off-diagonal links; above, entries carry
// pair_index and packedT holds all L links.  packedT orders each string's
// links by ascending pair field (a string's links have distinct pairs): at
// link step l the lanes of a wave then read nearby rows of G's row block,
// which the L1 and L2 serve far better than the canonical order's spread.
__global__ void k_links(int n, int ne, int64_t N, uint32_t* packed, uint32_t* packedT,
                        int32_t* abi4) {
  constexpr int kSortMax = kMaxActive * (kMaxActive / 2 + 1);  // links of a CASCI string
  int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= N) return;
  const int L = ne * (n - ne + 1);
  const bool sortT = packedT && L <= kSortMax;
  const bool fold = n <= kFoldMax;  // the gather's layout of G (see k_sigma_gather)
  const int nd = fold ? ne : 0;     // leading diagonal links left out of packedT
  uint32_t vs[kSortMax];
  uint64_t m = string_unrank(I, n, ne);
  int idx = 0;
  auto put = [&](uint32_t v) {
    if (packed) packed[I * L + idx] = v;
    if (sortT) vs[idx] = v;
    else if (packedT && idx >= nd) packedT[(idx - nd) * N + I] = v;
  };
  for (int o = 0; o < n; ++o)
    if (m >> o & 1) {
      put(pack_link((int)I, pair_index(o, o), 1));
      if (abi4) {
        int32_t* e = abi4 + (I * L + idx) * 4;
        e[0] = o; e[1] = o; e[2] = (int32_t)I; e[3] = 1;
      }
      ++idx;
    }
  for (int q = 0; q < n; ++q) {
    if (!(m >> q & 1)) continue;
    for (int p = 0; p < n; ++p) {
      if (m >> p & 1) continue;
      uint64_t r = (m & ~((uint64_t)1 << q)) | ((uint64_t)1 << p);
      int lo = p < q ? p : q, hi = p < q ? q : p;
      uint64_t between = (((uint64_t)1 << hi) - 1) & ~((((uint64_t)1 << lo) << 1) - 1);
      int sign = (__builtin_popcountll(m & between) & 1) ? -1 : 1;
      int64_t J = string_addr(r);
      put(pack_link((int)J, fold ? offdiag_index(hi, lo) : pair_index(hi, lo), sign));
      if (abi4) {
        int32_t* e = abi4 + (I * L + idx) * 4;
        e[0] = p; e[1] = q; e[2] = (int32_t)J; e[3] = sign;
      }
      ++idx;
    }
  }
  if (sortT)  // links nd..L-1 in ascending pair field (distinct within a string)
    for (int a = nd; a < L; ++a) {
      int rank = 0;
      for (int b = nd; b < L; ++b) rank += link_pair(vs[b]) < link_pair(vs[a]);
      packedT[rank * N + I] = vs[a];
    }
}

// One thread per string K: for every orbital pair a >= b the non-vanishing
// member of {E_ab K, E_ba K} (see pack_pair_entry).
__global__ void k_pair_table(int n, int ne, int64_t N, int32_t* out, int32_t* outT) {
  int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= N) return;
  const int npair = n * (n + 1) / 2;
  const uint64_t m = string_unrank(K, n, ne);
  int32_t* row = out + K * npair;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b <= a; ++b) {
      int32_t v = 0;
      const bool ia = m >> a & 1, ib = m >> b & 1;
      if (a == b) {
        if (ia) v = pack_pair_entry((int)K, 1);
      } else if (ia != ib) {
        // move the electron from the occupied one of (a, b) to the empty one
        const int q = ia ? a : b, p = ia ? b : a;
        const uint64_t r = (m & ~((uint64_t)1 << q)) | ((uint64_t)1 << p);
        const uint64_t between = (((uint64_t)1 << a) - 1) & ~((((uint64_t)1 << b) << 1) - 1);
        const int sign = (__builtin_popcountll(m & between) & 1) ? -1 : 1;
        v = pack_pair_entry((int)string_addr(r), sign);
      }
      row[a * (a + 1) / 2 + b] = v;
      outT[(int64_t)(a * (a + 1) / 2 + b) * N + K] = v;
    }
}

// ------------------------------------------------------- Hamiltonian set-up
// Frozen-core fold of the full-space Hamiltonian onto the active set A of one
// CASCI (frozen F = O \ A doubly occupied, all other orbitals deleted):
//   E_core = e_const + sum_{i in F} 2 h_ii + sum_{i,j in F} [2(ii|jj) - (ij|ji)]
//   h_eff_tu = h_tu + sum_{i in F} [2(tu|ii) - (ti|iu)]
// and the pair-space contraction matrix used by sigma = H c:
//   k_pq = h_eff_pq - 1/2 sum_{r in A} (pr|rq)
//   W_{ab,cd} = 1/2 (ab|cd) + (k_ab d_cd + d_ab k_cd) / (2N),  a>=b, c>=d,
// N = number of active electrons (the number operator acts as N on the CASCI
// space, which folds the one-body term into the single contraction).
struct ActiveSet {
  int n, na;
  int act[kMaxActive];
  int nf;
  int frz[kMaxOrb];
};

__device__ void build_item_hamiltonian(const ActiveSet& s, int M, const double* __restrict__ h1,
                                       const double* __restrict__ eri, double e_const, int nel,
                                       ItemHam* ham, double* W, int kpad) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int n = s.n;
  __shared__ double s_red[256];
  __shared__ double s_k[kMaxActive * kMaxActive];
  auto G = [&](int p, int q, int r, int u) -> double {
    return eri[(((size_t)p * M + q) * M + r) * M + u];
  };
  // frozen-core energy
  double e = 0.0;
  for (int x = t; x < s.nf * s.nf; x += nt) {
    int i = s.frz[x / s.nf], j = s.frz[x % s.nf];
    e += 2.0 * G(i, i, j, j) - G(i, j, j, i);
  }
  for (int x = t; x < s.nf; x += nt) e += 2.0 * h1[s.frz[x] * M + s.frz[x]];
  s_red[t] = e;
  __syncthreads();
  for (int w = nt / 2; w > 0; w >>= 1) {
    if (t < w) s_red[t] += s_red[t + w];
    __syncthreads();
  }
  if (t == 0) {
    ham->ecore = e_const + s_red[0];
    ham->eri = eri;
    ham->M = M;
    for (int i = 0; i < kMaxActive; ++i) ham->act[i] = i < n ? s.act[i] : 0;
  }
  // effective one-electron operator, Coulomb/exchange diagonals
  for (int x = t; x < n * n; x += nt) {
    int tt = x / n, uu = x % n;
    int p = s.act[tt], q = s.act[uu];
    double v = h1[p * M + q];
    for (int f = 0; f < s.nf; ++f) {
      int i = s.frz[f];
      v += 2.0 * G(p, q, i, i) - G(p, i, i, q);
    }
    ham->heff[tt * kMaxActive + uu] = v;
    ham->J[tt * kMaxActive + uu] = G(p, p, q, q);
    ham->K[tt * kMaxActive + uu] = G(p, q, q, p);
    double kv = v;
    for (int r = 0; r < n; ++r) kv -= 0.5 * G(p, s.act[r], s.act[r], q);
    s_k[tt * kMaxActive + uu] = kv;
  }
  __syncthreads();
  if (W) {
    const double inv2n = nel > 0 ? 0.5 / nel : 0.0;
    const int npair = n * (n + 1) / 2;
    for (int x = t; x < kpad * kpad; x += nt) {
      int ab = x / kpad, cd = x % kpad;
      double v = 0.0;
      if (ab < npair && cd < npair) {
        int a = 0;
        while ((a + 1) * (a + 2) / 2 <= ab) ++a;
        int b = ab - a * (a + 1) / 2;
        int c = 0;
        while ((c + 1) * (c + 2) / 2 <= cd) ++c;
        int d = cd - c * (c + 1) / 2;
        v = 0.5 * G(s.act[a], s.act[b], s.act[c], s.act[d]);
        if (c == d) v += inv2n * s_k[a * kMaxActive + b];
        if (a == b) v += inv2n * s_k[c * kMaxActive + d];
      }
      W[x] = v;
    }
  }
}

// One block per item: decode the tuple of bucket (order, nocc) from its index
// (lexicographic ranks of its occupied and virtual parts), form A = R u T and
// F = O \ A, and build the item's folded Hamiltonian and W.
__global__ void k_mbe_setup(MbeSpaces sp, const BucketDev* __restrict__ buckets, int nbucket,
                            const Item* __restrict__ items, const double* __restrict__ h1,
                            const double* __restrict__ eri, double e_const, ItemHam* hams,
                            double* warena, int32_t* tuple_pos, int max_order,
                            int32_t* act_out) {
  const int it = blockIdx.x;
  __shared__ ActiveSet s;
  if (threadIdx.x == 0) {
    int b = 0;
    while (b + 1 < nbucket && buckets[b + 1].item0 <= it) ++b;
    const BucketDev bk = buckets[b];
    int64_t local = it - bk.item0;
    int nv = bk.order - bk.nocc;
    int64_t cv = binom(sp.nXv, nv);
    int64_t ro = local / cv, rv = local % cv;
    int co[kMaxActive], cvv[kMaxActive];
    comb_lex_unrank(ro, bk.nocc, sp.nXo, co);
    comb_lex_unrank(rv, nv, sp.nXv, cvv);
    // active set: merge R, Xo[co], Xv[cvv] (all disjoint), sorted ascending
    int tmp[kMaxActive];
    int nt = 0;
    for (int i = 0; i < sp.nR; ++i) tmp[nt++] = sp.R[i];
    for (int i = 0; i < bk.nocc; ++i) tmp[nt++] = sp.Xo[co[i]];
    for (int i = 0; i < nv; ++i) tmp[nt++] = sp.Xv[cvv[i]];
    for (int i = 1; i < nt; ++i) {
      int v = tmp[i], j = i - 1;
      while (j >= 0 && tmp[j] > v) { tmp[j + 1] = tmp[j]; --j; }
      tmp[j + 1] = v;
    }
    s.n = nt;
    for (int i = 0; i < nt; ++i) s.act[i] = tmp[i];
    s.nf = 0;
    for (int i = 0; i < sp.nO; ++i) {
      int o = sp.O[i];
      bool in = false;
      for (int j = 0; j < nt; ++j) in |= (tmp[j] == o);
      if (!in) s.frz[s.nf++] = o;
    }
    s.na = sp.nocc_ref + bk.nocc;
    if (act_out)
      for (int i = 0; i < kMaxActive; ++i) act_out[it * kMaxActive + i] = i < nt ? tmp[i] : -1;
    if (tuple_pos) {
      // positions: occupied part (indices into Xo), then virtual part (into Xv)
      int32_t* tp = tuple_pos + (int64_t)it * (2 * max_order + 2);
      tp[0] = bk.nocc;
      tp[1] = nv;
      for (int i = 0; i < bk.nocc; ++i) tp[2 + i] = co[i];
      for (int i = 0; i < nv; ++i) tp[2 + bk.nocc + i] = cvv[i];
    }
  }
  __syncthreads();
  const Item& I = items[it];
  build_item_hamiltonian(s, sp.M, h1, eri, e_const, I.na + I.nb, &hams[I.ham],
                         I.ndet > 1 ? warena + I.woff : nullptr, I.kpad);
}

// Direct CASCI set-up: the whole given space is active (no frozen orbitals).
__global__ void k_casci_setup(int n, const double* const* h1s, const double* const* eris,
                              const double* ecores, const Item* __restrict__ items, ItemHam* hams,
                              double* warena) {
  const int it = blockIdx.x;
  __shared__ ActiveSet s;
  if (threadIdx.x == 0) {
    s.n = n;
    for (int i = 0; i < n; ++i) s.act[i] = i;
    s.nf = 0;
    s.na = items[it].na;
  }
  __syncthreads();
  const Item& I = items[it];
  build_item_hamiltonian(s, n, h1s[it], eris[it], ecores[it], I.na + I.nb, &hams[I.ham],
                         I.ndet > 1 ? warena + I.woff : nullptr, I.kpad);
}

// --------------------------------------------------------------- diagonal
// H_II - E_core = sum_{p in Ia u Ib} h_eff_pp + sum_{p<q in Ia} [(pp|qq)-(pq|qp)]
//               + same for Ib + sum_{p in Ia, q in Ib} (pp|qq)
__global__ void k_hdiag(const Item* __restrict__ items, const Work* __restrict__ work,
                        const ItemHam* __restrict__ hams, double* diag) {
  const Work wk = work[blockIdx.x];
  const Item& I = items[wk.item];
  const int64_t K = (int64_t)wk.begin * blockDim.x + threadIdx.x;
  if (K >= I.ndet) return;
  const ItemHam& H = hams[I.ham];
  uint64_t ma, mb;
  det_strings(I, K, ma, mb);
  double e = 0.0;
  for (uint64_t x = ma; x; x &= x - 1) {
    int p = __builtin_ctzll(x);
    e += H.heff[p * kMaxActive + p];
    for (uint64_t y = x & (x - 1); y; y &= y - 1) {
      int q = __builtin_ctzll(y);
      e += H.J[p * kMaxActive + q] - H.K[p * kMaxActive + q];
    }
    for (uint64_t y = mb; y; y &= y - 1) e += H.J[p * kMaxActive + __builtin_ctzll(y)];
  }
  for (uint64_t x = mb; x; x &= x - 1) {
    int p = __builtin_ctzll(x);
    e += H.heff[p * kMaxActive + p];
    for (uint64_t y = x & (x - 1); y; y &= y - 1) {
      int q = __builtin_ctzll(y);
      e += H.J[p * kMaxActive + q] - H.K[p * kMaxActive + q];
    }
  }
  diag[I.off + K] = e;
}

// ------------------------------------------------------------------ sigma
// sigma = (H - E_core) c by the Knowles-Handy / Olsen factorisation:
//   D+_ab[K] = <K| E_ab + E_ba |c>   (a > b),   D+_aa[K] = <K|E_aa|c>
//   G = W D+                          (the only dense step: FP64 MFMA)
//   sigma_I = sum over links E_xy I = s K of s G_pair(x,y)[K]
// Step 1+2 run fused in k_sigma_dgemm (D+ tile in LDS), step 3 in
// k_sigma_gather.  Both read the vector slot given by `slot` (>= 0: fixed
// slot, items with slot >= their guess count skip; -1: the item's newest).
typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ inline int vec_slot(const DavState& st, int slot) {
  return slot >= 0 ? slot : st.m - 1;
}
// f(std::integral_constant<int, M>{}) with M = m for m = 0..8 (returns
// true), else nothing (returns false): the Davidson passes loop over the
// subspace vectors with M known at compile time, so the loop unrolls without
// a branch per vector and a thread issues all of its loads at once.  Larger
// subspaces take the passes' generic loops.
template <class F>
__device__ inline bool with_space(int m, F&& f) {
  switch (m) {
    case 0: f(std::integral_constant<int, 0>{}); return true;
    case 1: f(std::integral_constant<int, 1>{}); return true;
    case 2: f(std::integral_constant<int, 2>{}); return true;
    case 3: f(std::integral_constant<int, 3>{}); return true;
    case 4: f(std::integral_constant<int, 4>{}); return true;
    case 5: f(std::integral_constant<int, 5>{}); return true;
    case 6: f(std::integral_constant<int, 6>{}); return true;
    case 7: f(std::integral_constant<int, 7>{}); return true;
    case 8: f(std::integral_constant<int, 8>{}); return true;
    default: return false;
  }
}
__device__ inline bool item_active(const DavState& st, int slot) {
  if (st.conv) return false;
  return slot < 0 || slot < st.nguess;
}

// Contraction G = W D+ on FP64 MFMA.  A tile is one alpha string Ka and TN
// consecutive beta strings; a workgroup keeps one beta block (TN strings)
// and walks down a range of alpha strings (tiles are numbered column-major:
// tile = block * Na + Ka).  A thread builds the same (pair, column) slots of
// D+ in every tile; their beta pair-table entries are loaded once per work
// unit, into registers for 32-column tiles of up to 10 orbitals (where the
// kernel still fits four waves per SIMD) and into LDS otherwise.  Per tile
// the c row of Ka is staged in LDS.  The alpha half of a D+ entry is
// wave-uniform: a scalar pair-table load and a coalesced row segment of c.
// D+ [pair][TN] (B operand) is staged in LDS, the wave's W rows (A operand)
// sit in registers.  G is stored [Ka][row][Kb], rows g_stride(Nb) long: up to
// kFoldMax orbitals the off-diagonal pairs (row offdiag_index), above every
// pair (row pair_index, k_sigma_dgemm_pairrows).
constexpr int64_t binom_c(int n, int k) {
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Up to kFoldMax orbitals the diagonal pairs kk need no row of G: E_kk only counts occupations, so
// their part of sigma, sum_k n_k(I) G_kk[I] with n_k(I) = n_k(Ia) + n_k(Ib),
// is summed in the contraction's epilogue and written to sigma, and the
// gather adds the off-diagonal links to it.  The contraction's output rows
// are the off-diagonal pairs a > b first (row offdiag_index(a, b), the row of
// G, which the gather's link tables carry), then padding, then the n
// diagonal pairs in the last n rows of the last 16-row block (row
// nrows - n + k: pair kk).  That block's wave, which sums the diagonal part,
// has few or no G rows to store, so the waves stay balanced.
// pair_index of output row r (nrows rows, n orbitals; -1: padding)
__device__ inline int out_row_pair(int r, int n, int nrows) {
  if (r >= nrows - n) return pair_index(r - (nrows - n), r - (nrows - n));
  if (r >= n * (n - 1) / 2) return -1;
  int a = 1;
  while ((a + 1) * a / 2 <= r) ++a;
  return pair_index(a, r - a * (a - 1) / 2);
}

// With 32-column tiles of up to 10 orbitals the pair-table entries stay in
// registers and the kernel is compiled for four waves per SIMD (128 registers
// per lane, accumulators included), which those shapes reach without
// spilling; larger shapes take the registers they need.  Active spaces of
// 11 or more orbitals run larger workgroups, since their LDS holds one or two
// workgroups per CU: 512 threads (two waves per SIMD) for 11-12 orbitals,
// 1024 (four per SIMD) for 13-14, where waves split a tile's output blocks
// by row block and column half.
// Active spaces of 8 or 9 orbitals have three 16-row blocks of G (36 or 45
// pairs padded to 48): their workgroups have three waves, one row block
// each, so that every wave of the CU issues MFMAs.
constexpr int dgemm_threads(int nact) {
  return nact >= 13 ? 1024 : nact >= 11 ? 512 : (nact == 8 || nact == 9) ? 192 : 256;
}
constexpr bool dgemm_reg_entries(int nact, int tn, int nt) {
  return (nt == 256 || nt == 192) && tn == 32 && nact <= 10;
}

template <int NACT, int TN, int NT = dgemm_threads(NACT)>
__global__ void __launch_bounds__(NT, dgemm_reg_entries(NACT, TN, NT) ? 4 : 1) k_sigma_dgemm(
    const Item* __restrict__ items, const Work* __restrict__ work,
    const double* __restrict__ warena, const double* __restrict__ V, int64_t ntot,
    double* __restrict__ Garena, double* __restrict__ Sarena, const DavState* __restrict__ st,
    int slot) {
  constexpr int NP = NACT * (NACT + 1) / 2;
  constexpr int KPAD = (NP + 15) / 16 * 16;
  constexpr int KS = (NP + 3) / 4;       // MFMA k-steps (4 pair rows per step)
  constexpr int KR = KS * 4;             // D+ rows held in LDS (zero beyond NP)
  constexpr int NRB = KPAD / 16;         // 16-row blocks of G
  constexpr int NW = NT / 64;            // waves per workgroup
  constexpr int NCB = TN / 16;           // 16-column blocks per tile
  constexpr int NCG = (NW >= 16 && NCB % 2 == 0) ? 2 : 1;  // column groups of waves
  constexpr int NRG = NW / NCG;          // row groups of waves
  constexpr int NCBW = NCB / NCG;        // column blocks per wave
  constexpr int RBW = (NRB + NRG - 1) / NRG;  // row blocks per wave
  constexpr int NSUB = NT / TN;          // row groups of the D+ build
  constexpr int NPER = (NP + NSUB - 1) / NSUB;
  constexpr int LDT = TN + 1;            // padded LDS row (doubles)
  constexpr int CMAX = (int)binom_c(NACT, NACT / 2);  // largest string count for NACT
  constexpr int CPT = (CMAX + NT - 1) / NT;           // c-row doubles per thread
  constexpr int TPT = (NP * TN + NT - 1) / NT;        // beta-table entries per thread
  constexpr bool EREG = dgemm_reg_entries(NACT, TN, NT);  // the launch-bounds rule
  constexpr int NO = NP - NACT;          // off-diagonal pairs: the rows of G
  static_assert(NACT <= kFoldMax, "larger active spaces take k_sigma_dgemm_pairrows");
  __shared__ double Ds[KR * LDT];
  __shared__ int32_t Tb[EREG ? 1 : NP * TN];
  __shared__ double Cr[CMAX];
  __shared__ uint32_t occB[TN];          // occupations of the work unit's beta strings

  const Work wk = work[blockIdx.x];
  const Item& I = items[wk.item];
  const DavState& S = st[wk.item];
  if (!item_active(S, slot)) return;
  const int vs = vec_slot(S, slot);
  const double* __restrict__ c = V + (int64_t)vs * ntot + I.off;
  double* __restrict__ G = Garena + I.goff;
  const int Na = I.Na, Nb = I.Nb;
  const int32_t* __restrict__ pA = I.pairA;
  const int32_t* __restrict__ pB = I.pairB;

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int col = t % TN;
  const int sub = (TN >= 64) ? __builtin_amdgcn_readfirstlane(t / TN) : t / TN;

  const int blk = wk.begin / Na;          // every work unit stays inside one beta block
  const int Kb0 = blk * TN;
  const int Kb = Kb0 + col;
  const double keep = Kb < Nb ? 1.0 : 0.0;  // ragged end of the row: zero columns
  const int Kbc = Kb < Nb ? Kb : Nb - 1;
  const double* __restrict__ ca = c + Kbc;  // alpha source of D+: ca[Ja * Nb]
  for (int x = t; x < TN; x += NT) occB[x] = Kb0 + x < Nb ? (uint32_t)ldg(I.strB + Kb0 + x) : 0u;

  // Row blocks rb = wrot + NRG r and column blocks cg NCBW .. of this wave.
  // When the 16-row blocks of G do not come in multiples of NRG some waves
  // have one block fewer; rotating the assignment by workgroup spreads those
  // idle slots over the SIMDs.
  const int cg = NCG == 1 ? 0 : wave / NRG;
  const int wrot = ((NCG == 1 ? wave : wave % NRG) + (int)blockIdx.x) % NRG;
  // W rows of this wave's row blocks, as MFMA A operands: lane l holds
  // W[rb*16 + l%16][ks*4 + l/16] (B operand: lane l holds D+[ks*4 + l/16][l%16])
  double wreg[RBW][KS];
  const double* __restrict__ W = warena + I.woff;
#pragma unroll
  for (int r = 0; r < RBW; ++r) {
    const int rb = wrot + NRG * r;
    const int wr = rb < NRB ? out_row_pair(rb * 16 + (lane & 15), NACT, KPAD) : -1;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      wreg[r][ks] = wr >= 0 ? ldg(W + wr * KPAD + ks * 4 + (lane >> 4)) : 0.0;
  }
  // This thread's beta pair-table entries: slot i is pair sub + NSUB i of
  // column col (x = t + NT i has x / TN = sub + NSUB i and x % TN = col),
  // the slots it writes in every tile's D+.  Then the zero padding rows of D+.
  static_assert(TPT == NPER, "one pair-table entry per D+ slot of a thread");
  // With EREG the entries stay in registers, packed: the Cr position jb of
  // slot i in byte i % 4 of jbp[i / 4], its sign and non-zero flag in bit i
  // of sgb and nzb (at most 10 orbitals: jb < 256).
  constexpr int NJP = (NPER + 3) / 4;
  uint32_t jbp[NJP], sgb = 0, nzb = 0;
#pragma unroll
  for (int q = 0; q < NJP; ++q) jbp[q] = 0;
#pragma unroll
  for (int i = 0; i < NPER; ++i) {
    const int ab = sub + NSUB * i;
    const int32_t e = ab < NP ? ldg(pB + ab * Nb + Kbc) : 0;
    if constexpr (EREG) {
      jbp[i / 4] |= (uint32_t)(e ? (e >> 1) - 1 : 0) << (8 * (i % 4));
      sgb |= (uint32_t)(e & 1) << i;
      nzb |= (uint32_t)(e != 0) << i;
    } else if (ab < NP) {
      Tb[t + NT * i] = e;
    }
  }
  for (int x = NP * LDT + t; x < KR * LDT; x += NT) Ds[x] = 0.0;

  // Software pipeline over the tiles of the work unit: the alpha pair-table
  // entries of tile i+1 are loaded while tile i builds D+, and the c row and
  // alpha-half values of tile i+1 while tile i runs its MFMAs.
  int32_t ea[NPER];   // alpha pair-table entries (only while their values are loaded)
  uint32_t sga = 0, nza = 0;  // their signs and non-zero flags, bit i
  double ga[NPER];    // c values they address (alpha half of D+)
  double cr[CPT];     // this thread's share of the c row Ka
  // The alpha entries are wave-uniform per row (scalar loads): with TN = 32
  // a wave covers the two rows 2*wave and 2*wave+1 of each row group.
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  auto load_entries = [&](int ka, int32_t (&e)[NPER]) {
    const int32_t* __restrict__ pa = pA + ka * NP;
#pragma unroll
    for (int i = 0; i < NPER; ++i) {
      if constexpr (TN >= 64) {
        const int ab = sub + NSUB * i;
        e[i] = ab < NP ? ldc(pa + ab) : 0;
      } else {
        static_assert(TN == 32, "tile width 32, 64 or 128");
        const int ab0 = 2 * wave_u + NSUB * i;
        const int32_t e0 = ab0 < NP ? ldc(pa + ab0) : 0;
        const int32_t e1 = ab0 + 1 < NP ? ldc(pa + ab0 + 1) : 0;
        e[i] = lane < 32 ? e0 : e1;
      }
    }
  };
  auto load_values = [&](int ka) {
    if constexpr (EREG) {
      sga = 0;
      nza = 0;
    }
#pragma unroll
    for (int i = 0; i < NPER; ++i) {
      ga[i] = ea[i] ? ldg(ca + ((ea[i] >> 1) - 1) * Nb) : 0.0;
      if constexpr (EREG) {
        sga |= (uint32_t)(ea[i] & 1) << i;
        nza |= (uint32_t)(ea[i] != 0) << i;
      }
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int x = t + NT * j;
      cr[j] = x < Nb ? ldg(c + ka * Nb + x) : 0.0;
    }
  };
  load_entries(wk.begin - blk * Na, ea);
  load_values(wk.begin - blk * Na);

  for (int tile = wk.begin; tile < wk.end; ++tile) {
    const int Ka = tile - blk * Na;              // uniform
    const bool more = tile + 1 < wk.end;
#pragma unroll
    for (int j = 0; j < CPT; ++j)
      if (t + NT * j < Nb) Cr[t + NT * j] = cr[j];
    // the next tile's alpha entries: for the register-entry kernels after the
    // D+ build (their registers are short), else ahead of it
    int32_t en[EREG ? 1 : NPER];
    if constexpr (!EREG) {
      if (more) {
        load_entries(Ka + 1, en);
      } else {
#pragma unroll
        for (int i = 0; i < NPER; ++i) en[i] = 0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NPER; ++i) {
      const int ab = sub + NSUB * i;
      if (ab < NP) {
        int jb;
        double fb;
        if constexpr (EREG) {
          jb = (jbp[i / 4] >> (8 * (i % 4))) & 0xFF;
          fb = (nzb >> i & 1) ? ((sgb >> i & 1) ? -keep : keep) : 0.0;
        } else {
          const int32_t e = Tb[t + NT * i];
          jb = e ? (e >> 1) - 1 : 0;
          fb = e ? ((e & 1) ? -keep : keep) : 0.0;
        }
        double fa;
        if constexpr (EREG) fa = (nza >> i & 1) ? ((sga >> i & 1) ? -keep : keep) : 0.0;
        else fa = ea[i] ? ((ea[i] & 1) ? -keep : keep) : 0.0;
        Ds[ab * LDT + col] = fa * ga[i] + fb * Cr[jb];
      }
    }
    __syncthreads();
    if (more) {
      if constexpr (EREG) {
        load_entries(Ka + 1, ea);
      } else {
#pragma unroll
        for (int i = 0; i < NPER; ++i) ea[i] = en[i];
      }
      load_values(Ka + 1);
    }
#pragma unroll
    for (int r = 0; r < RBW; ++r) {
      const int rb = wrot + NRG * r;
      if (rb >= NRB) continue;
      double4_t acc[NCBW];
#pragma unroll
      for (int cb2 = 0; cb2 < NCBW; ++cb2) acc[cb2] = (double4_t){0.0, 0.0, 0.0, 0.0};
      // B operands double-buffered in registers: the LDS reads of k-step
      // ks+1 are issued before the MFMAs of k-step ks
      double bq[2][NCBW];
      const double* bbase = Ds + (lane >> 4) * LDT + cg * NCBW * 16 + (lane & 15);
#pragma unroll
      for (int cb2 = 0; cb2 < NCBW; ++cb2) bq[0][cb2] = bbase[cb2 * 16];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        if (ks + 1 < KS) {
#pragma unroll
          for (int cb2 = 0; cb2 < NCBW; ++cb2)
            bq[(ks + 1) & 1][cb2] = bbase[(ks + 1) * 4 * LDT + cb2 * 16];
        }
#pragma unroll
        for (int cb2 = 0; cb2 < NCBW; ++cb2)
          acc[cb2] = __builtin_amdgcn_mfma_f64_16x16x4f64(wreg[r][ks], bq[ks & 1][cb2], acc[cb2],
                                                          0, 0, 0);
      }
      // instruction order for the scheduler: the first B reads, then per
      // k-step the next step's B reads (0x100: LDS read) ahead of this
      // step's MFMAs (0x008)
      __builtin_amdgcn_sched_group_barrier(0x100, NCBW, 0);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        if (ks + 1 < KS) __builtin_amdgcn_sched_group_barrier(0x100, NCBW, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, NCBW, 0);
      }
      const int Gs = g_stride(Nb);  // row stride of G
      double* __restrict__ Grow = G + (int64_t)Ka * NO * Gs;
#pragma unroll
      for (int cb2 = 0; cb2 < NCBW; ++cb2) {
        const int cl = (cg * NCBW + cb2) * 16 + (lane & 15);  // column in the tile
        const int Kc = Kb0 + cl;
        // gfx950 FP64 16x16x4 output layout: register v of lane l is row
        // l/16 + 4v, column l%16 of the 16x16 block
        if (rb == NRB - 1) {
          // the last block's rows 16 - NACT + k: the diagonal pairs, summed
          // into sigma with weights n_k(Ka) + n_k(Kb), lanes l/16 in a fixed order
          const uint32_t sa = (uint32_t)ldc(I.strA + Ka), sb = occB[cl];
          double pd = 0.0;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int k = (lane >> 4) + 4 * v - (16 - NACT);
            if (k >= 0) pd += (double)(((sa >> k) & 1) + ((sb >> k) & 1)) * acc[cb2][v];
          }
          pd += __shfl_xor(pd, 16, 64);
          pd += __shfl_xor(pd, 32, 64);
          if ((lane >> 4) == 0 && Kc < Nb)
            Sarena[(int64_t)vs * ntot + I.off + (int64_t)Ka * Nb + Kc] = pd;
        }
        if (Kc < Gs) {  // the row's padding too (zero: D+ is zero there), whole lines
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = rb * 16 + (lane >> 4) + 4 * v;
            if (row < NO) Grow[row * Gs + Kc] = acc[cb2][v];
          }
        }
      }
    }
    // No barrier here: the next tile's Cr stores follow this tile's second
    // barrier (every D+ read of Cr is done), and its D+ stores follow the
    // next first barrier (every MFMA read of Ds is done).
  }
}

// The contraction for active spaces of more than kFoldMax orbitals: G holds
// every pair row, [Ka][pair_index][Kb], diagonal pairs included, and the
// gather adds all links.  Their workgroups (512 and 1024 threads) have no
// register room for the diagonal epilogue of k_sigma_dgemm (measured: 3
// instead of 4 waves per SIMD at 11-12 orbitals, spills at 14), so they keep
// this layout.  Same tiles, D+ build and MFMA order as k_sigma_dgemm.
template <int NACT, int TN, int NT = dgemm_threads(NACT)>
__global__ void __launch_bounds__(NT, dgemm_reg_entries(NACT, TN, NT) ? 4 : 1) k_sigma_dgemm_pairrows(
    const Item* __restrict__ items, const Work* __restrict__ work,
    const double* __restrict__ warena, const double* __restrict__ V, int64_t ntot,
    double* __restrict__ Garena, const DavState* __restrict__ st, int slot) {
  constexpr int NP = NACT * (NACT + 1) / 2;
  constexpr int KPAD = (NP + 15) / 16 * 16;
  constexpr int KS = (NP + 3) / 4;       // MFMA k-steps (4 pair rows per step)
  constexpr int KR = KS * 4;             // D+ rows held in LDS (zero beyond NP)
  constexpr int NRB = KPAD / 16;         // 16-row blocks of G
  constexpr int NW = NT / 64;            // waves per workgroup
  constexpr int NCB = TN / 16;           // 16-column blocks per tile
  constexpr int NCG = (NW >= 16 && NCB % 2 == 0) ? 2 : 1;  // column groups of waves
  constexpr int NRG = NW / NCG;          // row groups of waves
  constexpr int NCBW = NCB / NCG;        // column blocks per wave
  constexpr int RBW = (NRB + NRG - 1) / NRG;  // row blocks per wave
  constexpr int NSUB = NT / TN;          // row groups of the D+ build
  constexpr int NPER = (NP + NSUB - 1) / NSUB;
  constexpr int LDT = TN + 1;            // padded LDS row (doubles)
  constexpr int CMAX = (int)binom_c(NACT, NACT / 2);  // largest string count for NACT
  constexpr int CPT = (CMAX + NT - 1) / NT;           // c-row doubles per thread
  constexpr int TPT = (NP * TN + NT - 1) / NT;        // beta-table entries per thread
  constexpr bool EREG = dgemm_reg_entries(NACT, TN, NT);  // the launch-bounds rule
  __shared__ double Ds[KR * LDT];
  __shared__ int32_t Tb[EREG ? 1 : NP * TN];
  __shared__ double Cr[CMAX];

  const Work wk = work[blockIdx.x];
  const Item& I = items[wk.item];
  const DavState& S = st[wk.item];
  if (!item_active(S, slot)) return;
  const int vs = vec_slot(S, slot);
  const double* __restrict__ c = V + (int64_t)vs * ntot + I.off;
  double* __restrict__ G = Garena + I.goff;
  const int Na = I.Na, Nb = I.Nb;
  const int32_t* __restrict__ pA = I.pairA;
  const int32_t* __restrict__ pB = I.pairB;

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int col = t % TN;
  const int sub = (TN >= 64) ? __builtin_amdgcn_readfirstlane(t / TN) : t / TN;

  const int blk = wk.begin / Na;          // every work unit stays inside one beta block
  const int Kb0 = blk * TN;
  const int Kb = Kb0 + col;
  const double keep = Kb < Nb ? 1.0 : 0.0;  // ragged end of the row: zero columns
  const int Kbc = Kb < Nb ? Kb : Nb - 1;
  const double* __restrict__ ca = c + Kbc;  // alpha source of D+: ca[Ja * Nb]

  // Row blocks rb = wrot + NRG r and column blocks cg NCBW .. of this wave.
  // When the 16-row blocks of G do not come in multiples of NRG some waves
  // have one block fewer; rotating the assignment by workgroup spreads those
  // idle slots over the SIMDs.
  const int cg = NCG == 1 ? 0 : wave / NRG;
  const int wrot = ((NCG == 1 ? wave : wave % NRG) + (int)blockIdx.x) % NRG;
  // W rows of this wave's row blocks, as MFMA A operands: lane l holds
  // W[rb*16 + l%16][ks*4 + l/16] (B operand: lane l holds D+[ks*4 + l/16][l%16])
  double wreg[RBW][KS];
  const double* __restrict__ W = warena + I.woff;
#pragma unroll
  for (int r = 0; r < RBW; ++r) {
    const int rb = wrot + NRG * r;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      wreg[r][ks] = (rb < NRB) ? ldg(W + (rb * 16 + (lane & 15)) * KPAD + ks * 4 + (lane >> 4))
                               : 0.0;
  }
  // This thread's beta pair-table entries: slot i is pair sub + NSUB i of
  // column col (x = t + NT i has x / TN = sub + NSUB i and x % TN = col),
  // the slots it writes in every tile's D+.  Then the zero padding rows of D+.
  static_assert(TPT == NPER, "one pair-table entry per D+ slot of a thread");
  int32_t eb[NPER];
#pragma unroll
  for (int i = 0; i < NPER; ++i) {
    const int ab = sub + NSUB * i;
    eb[i] = ab < NP ? ldg(pB + ab * Nb + Kbc) : 0;
  }
  if constexpr (!EREG) {
#pragma unroll
    for (int i = 0; i < NPER; ++i)
      if (sub + NSUB * i < NP) Tb[t + NT * i] = eb[i];
  }
  for (int x = NP * LDT + t; x < KR * LDT; x += NT) Ds[x] = 0.0;

  // Software pipeline over the tiles of the work unit: the alpha pair-table
  // entries of tile i+1 are loaded while tile i builds D+, and the c row and
  // alpha-half values of tile i+1 while tile i runs its MFMAs.
  int32_t ea[NPER];   // alpha pair-table entries of the current tile
  double ga[NPER];    // c values they address (alpha half of D+)
  double cr[CPT];     // this thread's share of the c row Ka
  // The alpha entries are wave-uniform per row (scalar loads): with TN = 32
  // a wave covers the two rows 2*wave and 2*wave+1 of each row group.
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  auto load_entries = [&](int ka, int32_t (&e)[NPER]) {
    const int32_t* __restrict__ pa = pA + ka * NP;
#pragma unroll
    for (int i = 0; i < NPER; ++i) {
      if constexpr (TN >= 64) {
        const int ab = sub + NSUB * i;
        e[i] = ab < NP ? ldc(pa + ab) : 0;
      } else {
        static_assert(TN == 32, "tile width 32, 64 or 128");
        const int ab0 = 2 * wave_u + NSUB * i;
        const int32_t e0 = ab0 < NP ? ldc(pa + ab0) : 0;
        const int32_t e1 = ab0 + 1 < NP ? ldc(pa + ab0 + 1) : 0;
        e[i] = lane < 32 ? e0 : e1;
      }
    }
  };
  auto load_values = [&](int ka) {
#pragma unroll
    for (int i = 0; i < NPER; ++i) ga[i] = ea[i] ? ldg(ca + ((ea[i] >> 1) - 1) * Nb) : 0.0;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int x = t + NT * j;
      cr[j] = x < Nb ? ldg(c + ka * Nb + x) : 0.0;
    }
  };
  load_entries(wk.begin - blk * Na, ea);
  load_values(wk.begin - blk * Na);

  for (int tile = wk.begin; tile < wk.end; ++tile) {
    const int Ka = tile - blk * Na;              // uniform
    const bool more = tile + 1 < wk.end;
#pragma unroll
    for (int j = 0; j < CPT; ++j)
      if (t + NT * j < Nb) Cr[t + NT * j] = cr[j];
    int32_t en[NPER];
    if (more) {
      load_entries(Ka + 1, en);
    } else {
#pragma unroll
      for (int i = 0; i < NPER; ++i) en[i] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NPER; ++i) {
      const int ab = sub + NSUB * i;
      if (ab < NP) {
        int32_t e;
        if constexpr (EREG) e = eb[i];
        else e = Tb[t + NT * i];
        const int jb = e ? (e >> 1) - 1 : 0;
        const double fa = ea[i] ? ((ea[i] & 1) ? -keep : keep) : 0.0;
        const double fb = e ? ((e & 1) ? -keep : keep) : 0.0;
        Ds[ab * LDT + col] = fa * ga[i] + fb * Cr[jb];
      }
    }
    __syncthreads();
    if (more) {
#pragma unroll
      for (int i = 0; i < NPER; ++i) ea[i] = en[i];
      load_values(Ka + 1);
    }
#pragma unroll
    for (int r = 0; r < RBW; ++r) {
      const int rb = wrot + NRG * r;
      if (rb >= NRB) continue;
      double4_t acc[NCBW];
#pragma unroll
      for (int cb2 = 0; cb2 < NCBW; ++cb2) acc[cb2] = (double4_t){0.0, 0.0, 0.0, 0.0};
      // B operands double-buffered in registers: the LDS reads of k-step
      // ks+1 are issued before the MFMAs of k-step ks
      double bq[2][NCBW];
      const double* bbase = Ds + (lane >> 4) * LDT + cg * NCBW * 16 + (lane & 15);
#pragma unroll
      for (int cb2 = 0; cb2 < NCBW; ++cb2) bq[0][cb2] = bbase[cb2 * 16];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        if (ks + 1 < KS) {
#pragma unroll
          for (int cb2 = 0; cb2 < NCBW; ++cb2)
            bq[(ks + 1) & 1][cb2] = bbase[(ks + 1) * 4 * LDT + cb2 * 16];
        }
#pragma unroll
        for (int cb2 = 0; cb2 < NCBW; ++cb2)
          acc[cb2] = __builtin_amdgcn_mfma_f64_16x16x4f64(wreg[r][ks], bq[ks & 1][cb2], acc[cb2],
                                                          0, 0, 0);
      }
      // instruction order for the scheduler: the first B reads, then per
      // k-step the next step's B reads (0x100: LDS read) ahead of this
      // step's MFMAs (0x008)
      __builtin_amdgcn_sched_group_barrier(0x100, NCBW, 0);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        if (ks + 1 < KS) __builtin_amdgcn_sched_group_barrier(0x100, NCBW, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, NCBW, 0);
      }
      const int Gs = g_stride(Nb);  // row stride of G
      double* __restrict__ Grow = G + (int64_t)Ka * NP * Gs;
#pragma unroll
      for (int cb2 = 0; cb2 < NCBW; ++cb2) {
        const int Kc = Kb0 + (cg * NCBW + cb2) * 16 + (lane & 15);
        if (Kc < Gs) {  // the row's padding too (zero: D+ is zero there), whole lines
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            // gfx950 FP64 16x16x4 output layout: register v of lane l is
            // row l/16 + 4v, column l%16 of the 16x16 block
            // non-temporal: at 11-14 orbitals G (a 1-3 MB row block per
            // alpha string) streams through the caches without reuse before
            // the gather, and cached stores only evict c and the tables
            const int row = rb * 16 + (lane >> 4) + 4 * v;
            if (row < NP) __builtin_nontemporal_store(acc[cb2][v], &Grow[row * Gs + Kc]);
          }
        }
      }
    }
    // No barrier here: the next tile's Cr stores follow this tile's second
    // barrier (every D+ read of Cr is done), and its D+ stores follow the
    // next first barrier (every MFMA read of Ds is done).
  }
}

// The same contraction on flattened tiles, for active spaces of at most 9
// orbitals (short beta strings, where a tile of one alpha string leaves the
// last beta block mostly empty): a tile is TN consecutive determinants
// K = Ka Nb + Kb of one item and may cross alpha strings, so only an item's
// last tile is ragged.  The whole beta pair table of the item is staged in LDS
// once per work unit, and per tile the c rows it spans (a contiguous stretch of
// c); the alpha pair entries and the alpha-half c values are per-lane loads,
// fetched one tile ahead.  D+ and the MFMA contraction are formed from
// the same operands in the same order as in k_sigma_dgemm, so G is identical.
// Work units hold ranges of flat tile numbers of one item.
template <int NACT, int TN>
__global__ void __launch_bounds__(256) k_sigma_dgemm_flat(const Item* __restrict__ items,
                                                          const Work* __restrict__ work,
                                                          const double* __restrict__ warena,
                                                          const double* __restrict__ V,
                                                          int64_t ntot,
                                                          double* __restrict__ Garena,
                                                          double* __restrict__ Sarena,
                                                          const DavState* __restrict__ st,
                                                          int slot) {
  static_assert(NACT <= 9, "flattened tiles stage the whole beta pair table");
  constexpr int NP = NACT * (NACT + 1) / 2;
  constexpr int KPAD = (NP + 15) / 16 * 16;
  constexpr int KS = (NP + 3) / 4;
  constexpr int KR = KS * 4;
  constexpr int NRB = KPAD / 16;
  constexpr int RBW = (NRB + 3) / 4;
  constexpr int NCB = TN / 16;
  constexpr int NSUB = 256 / TN;
  constexpr int NPER = (NP + NSUB - 1) / NSUB;
  constexpr int LDT = TN + 1;
  constexpr int CMAX = (int)binom_c(NACT, NACT / 2);
  constexpr int CRMAX = TN + 2 * CMAX;                 // c rows a tile can touch
  constexpr int CPT = (CRMAX + 255) / 256;
  constexpr int NO = NP - NACT;  // off-diagonal pairs: the rows of G
  static_assert(NACT <= kFoldMax, "flattened tiles sum the diagonal part themselves");
  __shared__ double Ds[KR * LDT];
  __shared__ int32_t Tb[NP * CMAX];  // beta pair table [pair][Kb]
  __shared__ double Cr[CRMAX];       // c rows Ka_lo .. Ka_hi of the tile

  const Work wk = work[blockIdx.x];
  const Item& I = items[wk.item];
  const DavState& S = st[wk.item];
  if (!item_active(S, slot)) return;
  const int vs = vec_slot(S, slot);
  const double* __restrict__ c = V + (int64_t)vs * ntot + I.off;
  double* __restrict__ G = Garena + I.goff;
  const int Nb = I.Nb;
  const int nd = (int)I.ndet;
  const int32_t* __restrict__ pA = I.pairA;
  const int32_t* __restrict__ pB = I.pairB;

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int col = t % TN;
  const int sub = (TN >= 64) ? __builtin_amdgcn_readfirstlane(t / TN) : t / TN;
  const int wrot = (wave + (int)blockIdx.x) & 3;
  double wreg[RBW][KS];
  const double* __restrict__ W = warena + I.woff;
#pragma unroll
  for (int r = 0; r < RBW; ++r) {
    const int rb = wrot + 4 * r;
    const int wr = rb < NRB ? out_row_pair(rb * 16 + (lane & 15), NACT, KPAD) : -1;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      wreg[r][ks] = wr >= 0 ? ldg(W + wr * KPAD + ks * 4 + (lane >> 4)) : 0.0;
  }
  for (int x = t; x < NP * Nb; x += 256) Tb[x] = ldg(pB + x);
  for (int x = NP * LDT + t; x < KR * LDT; x += 256) Ds[x] = 0.0;
  __syncthreads();

  // column position of this thread in a tile (past the item's end: the last
  // determinant, with weight zero)
  auto colpos = [&](int tile, int& ka, int& kb, double& kp) {
    int k = tile * TN + col;
    kp = k < nd ? 1.0 : 0.0;
    if (k >= nd) k = nd - 1;
    ka = k / Nb;
    kb = k - ka * Nb;
  };
  // first alpha string of a tile (its c rows are staged from there)
  auto row_lo = [&](int tile) { return (tile * TN) / Nb; };
  int32_t ea[NPER];  // alpha pair-table entries of the tile
  double ga[NPER];   // the c values they address (alpha half of D+)
  double cr[CPT];    // this thread's share of the tile's c rows
  auto load_entries = [&](int ka, int32_t (&xa)[NPER]) {
#pragma unroll
    for (int i = 0; i < NPER; ++i) {
      const int ab = sub + NSUB * i;
      xa[i] = ab < NP ? ldg(pA + ka * NP + ab) : 0;
    }
  };
  auto load_values = [&](int tile, int kb) {
#pragma unroll
    for (int i = 0; i < NPER; ++i) ga[i] = ea[i] ? ldg(c + ((ea[i] >> 1) - 1) * Nb + kb) : 0.0;
    const int lo = row_lo(tile) * Nb;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int x = lo + t + 256 * j;
      cr[j] = (t + 256 * j < CRMAX && x < nd) ? ldg(c + x) : 0.0;
    }
  };
  int ka, kb;
  double keep;
  colpos(wk.begin, ka, kb, keep);
  load_entries(ka, ea);
  load_values(wk.begin, kb);

  for (int tile = wk.begin; tile < wk.end; ++tile) {
    const bool more = tile + 1 < wk.end;
    int kan = 0, kbn = 0;
    double keepn = 0.0;
    int32_t ean[NPER];
#pragma unroll
    for (int j = 0; j < CPT; ++j)
      if (t + 256 * j < CRMAX) Cr[t + 256 * j] = cr[j];
    if (more) {
      colpos(tile + 1, kan, kbn, keepn);
      load_entries(kan, ean);
    } else {
#pragma unroll
      for (int i = 0; i < NPER; ++i) ean[i] = 0;
    }
    __syncthreads();
    const int crow = (ka - row_lo(tile)) * Nb;  // this column's c row in Cr
#pragma unroll
    for (int i = 0; i < NPER; ++i) {
      const int ab = sub + NSUB * i;
      if (ab < NP) {
        const int32_t eb = Tb[ab * Nb + kb];
        const int jb = eb ? (eb >> 1) - 1 : 0;
        const double fa = ea[i] ? ((ea[i] & 1) ? -keep : keep) : 0.0;
        const double fb = eb ? ((eb & 1) ? -keep : keep) : 0.0;
        Ds[ab * LDT + col] = fa * ga[i] + fb * Cr[crow + jb];
      }
    }
    __syncthreads();
    if (more) {
#pragma unroll
      for (int i = 0; i < NPER; ++i) ea[i] = ean[i];
      ka = kan;
      kb = kbn;
      keep = keepn;
      load_values(tile + 1, kb);
    }
#pragma unroll
    for (int r = 0; r < RBW; ++r) {
      const int rb = wrot + 4 * r;
      if (rb >= NRB) continue;
      double4_t acc[NCB];
#pragma unroll
      for (int cb2 = 0; cb2 < NCB; ++cb2) acc[cb2] = (double4_t){0.0, 0.0, 0.0, 0.0};
      double bq[2][NCB];
      const double* bbase = Ds + (lane >> 4) * LDT + (lane & 15);
#pragma unroll
      for (int cb2 = 0; cb2 < NCB; ++cb2) bq[0][cb2] = bbase[cb2 * 16];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        if (ks + 1 < KS) {
#pragma unroll
          for (int cb2 = 0; cb2 < NCB; ++cb2)
            bq[(ks + 1) & 1][cb2] = bbase[(ks + 1) * 4 * LDT + cb2 * 16];
        }
#pragma unroll
        for (int cb2 = 0; cb2 < NCB; ++cb2)
          acc[cb2] = __builtin_amdgcn_mfma_f64_16x16x4f64(wreg[r][ks], bq[ks & 1][cb2], acc[cb2],
                                                          0, 0, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x100, NCB, 0);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        if (ks + 1 < KS) __builtin_amdgcn_sched_group_barrier(0x100, NCB, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, NCB, 0);
      }
#pragma unroll
      for (int cb2 = 0; cb2 < NCB; ++cb2) {
        const int Kc = tile * TN + cb2 * 16 + (lane & 15);
        const int Kq = Kc < nd ? Kc : nd - 1;
        const int kac = Kq / Nb, kbc = Kq - kac * Nb;
        if (rb == NRB - 1) {  // the diagonal pairs' part of sigma, as in k_sigma_dgemm
          const uint32_t sa = (uint32_t)ldg(I.strA + kac), sb = (uint32_t)ldg(I.strB + kbc);
          double pd = 0.0;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int k = (lane >> 4) + 4 * v - (16 - NACT);
            if (k >= 0) pd += (double)(((sa >> k) & 1) + ((sb >> k) & 1)) * acc[cb2][v];
          }
          pd += __shfl_xor(pd, 16, 64);
          pd += __shfl_xor(pd, 32, 64);
          if ((lane >> 4) == 0 && Kc < nd) Sarena[(int64_t)vs * ntot + I.off + Kc] = pd;
        }
        if (Kc < nd) {
          double* __restrict__ Grow = G + (int64_t)kac * NO * g_stride(Nb) + kbc;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = rb * 16 + (lane >> 4) + 4 * v;
            if (row < NO) Grow[row * g_stride(Nb)] = acc[cb2][v];
          }
        }
      }
    }
    // No barrier here: the next tile's Cr stores follow this tile's second
    // barrier (every D+ read of Cr is done), and its D+ stores follow the
    // next first barrier (every MFMA read of Ds is done).
  }
}

// sigma_I = sum_{links (x,y,J,s) of Ia} s G_xy[J, Ib] + sum_{links of Ib} s G_xy[Ia, J].
// Up to kFoldMax orbitals the contraction wrote the diagonal links' part to
// sigma beforehand, G holds the off-diagonal rows and this adds the
// off-diagonal links (their entries carry G's row offdiag_index(x, y));
// above, it sums every link over G's pair_index rows.
// One wave per 64-determinant segment of one alpha row (segments are
// row-aligned), so the alpha string and its links are wave-uniform (scalar
// loads) and the alpha-part reads of G are coalesced rows.  Work units run
// in reverse order: the contraction wrote G in unit order, so the part it
// wrote last, still in the last-level cache, is read first.
__global__ void __launch_bounds__(256) k_sigma_gather(const Item* __restrict__ items,
                                                      const Work* __restrict__ work,
                                                      const double* __restrict__ Garena,
                                                      double* __restrict__ Sarena, int64_t ntot,
                                                      const DavState* __restrict__ st, int slot) {
  const Work wk = work[gridDim.x - 1 - blockIdx.x];
  const Item& I = items[wk.item];
  const DavState& S = st[wk.item];
  if (!item_active(S, slot)) return;
  const int vs = vec_slot(S, slot);
  const int Nb = I.Nb;
  const int segs = (Nb + 63) >> 6;  // segments per alpha row
  const int seg = __builtin_amdgcn_readfirstlane(wk.begin * 4 + (threadIdx.x >> 6));
  if (seg >= wk.end) return;
  const int Ka = __builtin_amdgcn_readfirstlane(seg / segs);
  const int Kb = (seg % segs) * 64 + (threadIdx.x & 63);
  if (Kb >= Nb) return;
  const double* __restrict__ G = Garena + I.goff;
  const int Gs = g_stride(Nb);  // row stride of G
  const int La = I.La, Lb = I.Lb;
  double acc0 = 0.0, acc1 = 0.0;
  // up to kFoldMax orbitals the contraction summed the diagonal links' part
  // and G holds the off-diagonal rows; otherwise G holds every pair row
  const bool fold = I.n <= kFoldMax;
  const int np = fold ? I.npair - I.n : I.npair;  // rows of G per alpha string
  const uint32_t* __restrict__ la = I.linkA + Ka * La;
  const double* __restrict__ Gcol = G + Kb;  // G[(Ja * npair + pair) * Gs + Kb]
  int l = fold ? I.na : 0;  // the first na links are the diagonal ones
  for (; l + 3 < La; l += 4) {
    const uint32_t e0 = ldc(la + l), e1 = ldc(la + l + 1), e2 = ldc(la + l + 2), e3 = ldc(la + l + 3);
    const double g0 = ldg(Gcol + (int64_t)(link_addr(e0) * np + link_pair(e0)) * Gs);
    const double g1 = ldg(Gcol + (int64_t)(link_addr(e1) * np + link_pair(e1)) * Gs);
    const double g2 = ldg(Gcol + (int64_t)(link_addr(e2) * np + link_pair(e2)) * Gs);
    const double g3 = ldg(Gcol + (int64_t)(link_addr(e3) * np + link_pair(e3)) * Gs);
    acc0 += link_sign(e0) * g0 + link_sign(e2) * g2;
    acc1 += link_sign(e1) * g1 + link_sign(e3) * g3;
  }
  for (; l < La; ++l) {
    const uint32_t e0 = ldc(la + l);
    acc0 += link_sign(e0) * ldg(Gcol + (int64_t)(link_addr(e0) * np + link_pair(e0)) * Gs);
  }
  const int Lo = fold ? Lb - I.nb : Lb;  // the links held in linkBT
  const uint32_t* __restrict__ lb = I.linkBT + Kb;               // link l of Kb: lb[l * Nb]
  const double* __restrict__ Grow = G + (int64_t)Ka * np * Gs;  // G[(Ka * npair + pair) * Gs + Jb]
  l = 0;
  for (; l + 3 < Lo; l += 4) {
    const uint32_t e0 = ldg(lb + l * Nb), e1 = ldg(lb + (l + 1) * Nb), e2 = ldg(lb + (l + 2) * Nb),
                   e3 = ldg(lb + (l + 3) * Nb);
    const double g0 = ldg(Grow + link_pair(e0) * Gs + link_addr(e0));
    const double g1 = ldg(Grow + link_pair(e1) * Gs + link_addr(e1));
    const double g2 = ldg(Grow + link_pair(e2) * Gs + link_addr(e2));
    const double g3 = ldg(Grow + link_pair(e3) * Gs + link_addr(e3));
    acc0 += link_sign(e0) * g0 + link_sign(e2) * g2;
    acc1 += link_sign(e1) * g1 + link_sign(e3) * g3;
  }
  for (; l < Lo; ++l) {
    const uint32_t e0 = ldg(lb + l * Nb);
    acc0 += link_sign(e0) * ldg(Grow + link_pair(e0) * Gs + link_addr(e0));
  }
  double* __restrict__ out = Sarena + (int64_t)vs * ntot + I.off + (int64_t)Ka * Nb + Kb;
  if (fold) *out += acc0 + acc1;
  else *out = acc0 + acc1;
}

// ------------------------------------------------------ input validation
// Finiteness and permutational symmetry of the MO integrals, on the device
// (no host copy of the M^4 tensor): each element is compared with its
// partners h_qp, and (qp|rs), (pq|sr), (rs|pq), to 1e-12 times the larger of
// 1 and the two magnitudes.  Bits of *flags (integer atomics): 1 h not finite,
// 2 h not symmetric, 4 eri not finite, 8 eri lacks the 8-fold symmetry.
__global__ void k_check_integrals(const double* __restrict__ h1, const double* __restrict__ eri,
                                  int M, int* flags) {
  const int64_t n1 = (int64_t)M * M, n2 = n1 * n1;
  int f = 0;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n1 + n2;
       x += (int64_t)gridDim.x * blockDim.x) {
    auto close = [](double a, double b) {
      const double sc = fmax(1.0, fmax(fabs(a), fabs(b)));
      return fabs(a - b) <= 1e-12 * sc;
    };
    if (x < n1) {
      const int p = (int)(x / M), q = (int)(x % M);
      const double a = h1[x];
      if (!isfinite(a)) f |= 1;
      else if (!close(a, h1[(int64_t)q * M + p])) f |= 2;
    } else {
      const int64_t y = x - n1;
      const int s = (int)(y % M), r = (int)(y / M % M), q = (int)(y / n1 % M), p = (int)(y / n1 / M);
      const double a = eri[y];
      auto at = [&](int i, int j, int k, int l) { return eri[(((int64_t)i * M + j) * M + k) * M + l]; };
      if (!isfinite(a)) f |= 4;
      else if (!close(a, at(q, p, r, s)) || !close(a, at(p, q, s, r)) || !close(a, at(r, s, p, q)))
        f |= 8;
    }
  }
  if (f) atomicOr(flags, f);
}

void launch_check_integrals(const double* h1, const double* eri, int M, int* flags,
                            hipStream_t s) {
  const int64_t n = (int64_t)M * M * (1 + (int64_t)M * M);
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_check_integrals, dim3((int)b), dim3(256), 0, s, h1, eri, M, flags);
}

// ------------------------------------------------- point-group blocked sigma
// The contraction of one pair class s on the determinants of irrep G^s:
// G_s = W_s D+_s on FP64 MFMA.  A work unit is (item, class s, alpha irrep
// a' of the irrep-G^s space) and a range of tiles of that block; a tile is
// one alpha string ka (local to irrep a') and TN consecutive beta strings of
// irrep b' = a'^G^s, numbered column-major (tile = block * nac[a'] + ka) so
// a unit stays inside one beta block.  D+ rows are the class's pairs,
// zero-padded to NPC.  The alpha half of a D+ entry reads c in CI block a'^s
// (beta irrep b', rows of nbc[b']), the beta half in block a' (rows of
// nbc[a'^G]).  Work.pad_ = s * 8 + a'.  Classes of up to 48 pairs take
// 64-column tiles with one 16-column block per wave (every wave busy however
// few row blocks the class has); larger ones 32-column tiles with row blocks
// dealt over the waves.
int sym_tile(int npc) { return npc <= 48 ? 64 : 32; }

template <int NPC, int TN>
__global__ void __launch_bounds__(256) k_sigma_sym_dgemm(
    const Item* __restrict__ items, const Work* __restrict__ work,
    const double* __restrict__ warena, const double* __restrict__ V, int64_t ntot,
    double* __restrict__ Garena, const DavState* __restrict__ st, int slot) {
  constexpr int KS = NPC / 4;       // MFMA k-steps
  constexpr int NRB = NPC / 16;     // 16-row blocks of G_s
  constexpr int NCB = TN / 16;
  constexpr bool COL = NCB == 4;    // wave w computes column block w, every row block
  constexpr int RBW = COL ? NRB : (NRB + 3) / 4;
  constexpr int LDT = TN + 1;
  __shared__ double Ds[NPC * LDT];
  __shared__ int32_t pl[NPC];       // class pair -> pair index (W row / column)

  const Work wk = work[blockIdx.x];
  const Item& I = items[wk.item];
  const DavState& S = st[wk.item];
  if (!item_active(S, slot)) return;
  const SymInfo& Y = *I.sym;
  const int vs = vec_slot(S, slot);
  const double* __restrict__ c = V + (int64_t)vs * ntot + I.off;
  const int s = wk.pad_ >> 3, ap = wk.pad_ & 7;
  const int G = Y.wfn;
  const int bp = ap ^ G ^ s;          // beta irrep of the tile
  const int nps = Y.cls0[s + 1] - Y.cls0[s];
  const int j0 = Y.cls0[s];
  const int NA = Y.nac[ap], NB = Y.nbc[bp];
  const int NBa = Y.nbc[ap ^ G];      // row length of CI block a'
  const double* __restrict__ csrcA = c + Y.blk[ap ^ s];  // block a'^s: rows of NB
  const double* __restrict__ csrcB = c + Y.blk[ap];      // block a': rows of NBa
  const int32_t* __restrict__ pA = I.pairA + (int64_t)Y.na0[ap] * Y.npair + j0;
  const int32_t* __restrict__ pB = I.pairB + (int64_t)j0 * I.Nb + Y.nb0[bp];
  double* __restrict__ G_s = Garena + I.goff + Y.gofs[s][ap];
  const int kpad = I.kpad;
  const double* __restrict__ W = warena + I.woff;

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  for (int i = t; i < NPC; i += 256) pl[i] = i < nps ? Y.pair_of[j0 + i] : -1;
  __syncthreads();
  const int wrot = (wave + (int)blockIdx.x) & 3;
  double wreg[RBW][KS];
#pragma unroll
  for (int r = 0; r < RBW; ++r) {
    const int rb = COL ? r : wrot + 4 * r;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int row = rb * 16 + (lane & 15), col = ks * 4 + (lane >> 4);
      wreg[r][ks] = (rb < NRB && row < nps && col < nps)
                        ? ldg(W + (int64_t)pl[row] * kpad + pl[col]) : 0.0;
    }
  }
  const int blk = wk.begin / NA;
  const int kb0 = blk * TN;
  // Classes of up to 32 pairs: this thread builds the D+ slots (class pair
  // sub + NSUB k, column col) of every tile of the unit; their beta
  // pair-table entries depend on the column only, so they are loaded once
  // per unit, and the alpha entries are wave-uniform per pair row (scalar
  // loads).  Larger classes build D+ element by element (registers for the
  // slots would cost them occupancy).
  constexpr bool SLOTS = NPC <= 32;
  constexpr int NSUB = 256 / TN;
  constexpr int NPER = SLOTS ? (NPC + NSUB - 1) / NSUB : 1;
  const int col = t % TN;
  const int sub = TN >= 64 ? __builtin_amdgcn_readfirstlane(t / TN) : t / TN;
  const int kb = kb0 + col;
  const bool live = kb < NB;
  const int kbc = live ? kb : NB - 1;
  int32_t eb[NPER];
  int32_t ea[NPER];
  double ga[NPER], gb[NPER];
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  auto load_tile = [&](int ka) {
    const int32_t* __restrict__ pa = pA + (int64_t)ka * Y.npair;
    const double* __restrict__ crow = csrcB + (int64_t)ka * NBa;
#pragma unroll
    for (int k = 0; k < NPER; ++k) {
      if constexpr (TN >= 64) {
        const int i = sub + NSUB * k;
        ea[k] = (i < nps) ? ldc(pa + i) : 0;
      } else {
        const int i0 = 2 * wave_u + NSUB * k;
        const int32_t e0 = i0 < nps ? ldc(pa + i0) : 0;
        const int32_t e1 = i0 + 1 < nps ? ldc(pa + i0 + 1) : 0;
        ea[k] = lane < 32 ? e0 : e1;
      }
      ga[k] = ea[k] ? ldg(csrcA + (int64_t)((ea[k] >> 1) - 1) * NB + kbc) : 0.0;
      gb[k] = eb[k] ? ldg(crow + ((eb[k] >> 1) - 1)) : 0.0;
    }
  };
  if constexpr (SLOTS) {
#pragma unroll
    for (int k = 0; k < NPER; ++k) {
      const int i = sub + NSUB * k;
      eb[k] = (i < nps && live) ? ldg(pB + (int64_t)i * I.Nb + kbc) : 0;
    }
  }
  for (int tile = wk.begin; tile < wk.end; ++tile) {
    const int ka = tile - blk * NA;
    // D+ tile [NPC][TN]: class pair i, column kb0 + col
    if constexpr (SLOTS) {
      load_tile(ka);
#pragma unroll
      for (int k = 0; k < NPER; ++k) {
        const int i = sub + NSUB * k;
        if (i < NPC) {
          const double fa = (ea[k] && live) ? ((ea[k] & 1) ? -1.0 : 1.0) : 0.0;
          const double fb = eb[k] ? ((eb[k] & 1) ? -1.0 : 1.0) : 0.0;
          Ds[i * LDT + col] = fa * ga[k] + fb * gb[k];
        }
      }
    } else {
      for (int x = t; x < NPC * TN; x += 256) {
        const int i = x / TN, cx = x % TN, kx = kb0 + cx;
        double v = 0.0;
        if (i < nps && kx < NB) {
          const int32_t e1 = ldg(pA + (int64_t)ka * Y.npair + i);
          if (e1) {
            const double cv = ldg(csrcA + (int64_t)((e1 >> 1) - 1) * NB + kx);
            v += (e1 & 1) ? -cv : cv;
          }
          const int32_t e2 = ldg(pB + (int64_t)i * I.Nb + kx);
          if (e2) {
            const double cv = ldg(csrcB + (int64_t)ka * NBa + ((e2 >> 1) - 1));
            v += (e2 & 1) ? -cv : cv;
          }
        }
        Ds[i * LDT + cx] = v;
      }
    }
    __syncthreads();
    // G rows are written with non-temporal stores: the class's G block is
    // not re-read before the gather (8 x CAS(14,14) in A_g: 59.8 -> 56.4 ms)
    double* __restrict__ Grows = G_s + (int64_t)ka * nps * NB;
    if constexpr (COL) {
      // this wave: columns kb0 + 16 wave .. + 15, every row block
      const double* bbase = Ds + (lane >> 4) * LDT + wave * 16 + (lane & 15);
      double4_t acc[NRB];
#pragma unroll
      for (int r = 0; r < NRB; ++r) acc[r] = (double4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const double bv = bbase[ks * 4 * LDT];
#pragma unroll
        for (int r = 0; r < NRB; ++r)
          acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(wreg[r][ks], bv, acc[r], 0, 0, 0);
      }
      const int kc = kb0 + wave * 16 + (lane & 15);
      if (kc < NB) {
#pragma unroll
        for (int r = 0; r < NRB; ++r)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            // register v of lane l: row l/16 + 4v, column l%16 of the block
            const int row = r * 16 + (lane >> 4) + 4 * v;
            if (row < nps) __builtin_nontemporal_store(acc[r][v], &Grows[(int64_t)row * NB + kc]);
          }
      }
    } else {
#pragma unroll
      for (int r = 0; r < RBW; ++r) {
        const int rb = wrot + 4 * r;
        if (rb >= NRB) continue;
        double4_t acc[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[cb] = (double4_t){0.0, 0.0, 0.0, 0.0};
        const double* bbase = Ds + (lane >> 4) * LDT + (lane & 15);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
            acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(wreg[r][ks],
                                                           bbase[ks * 4 * LDT + cb * 16], acc[cb],
                                                           0, 0, 0);
        }
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const int kc = kb0 + cb * 16 + (lane & 15);
          if (kc < NB) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = rb * 16 + (lane >> 4) + 4 * v;
              if (row < nps) __builtin_nontemporal_store(acc[cb][v], &Grows[(int64_t)row * NB + kc]);
            }
          }
        }
      }
    }
    __syncthreads();  // every MFMA read of Ds is done before the next tile's build
  }
}

// sigma_I = sum over links of I of sign * G_s[K], blocked layout: one thread per
// determinant I = (a, ia, ib) of irrep G (b = a^G).  An alpha link of ia
// (class-sorted pair j of class s, string Ja local to irrep a^s) reads G_s in
// block a^s, row (Ja, j - cls0[s]), column ib; a beta link of ib (string Jb
// local to irrep b^s) reads G_s in block a, row (ia, j - cls0[s]), column Jb.
// The class tables are staged in LDS; beta links come from the link-major
// table linkBT [Lb][Nb] (consecutive threads read consecutive entries).
// Work units: 256 consecutive determinants of one item (Work.begin).
__global__ void __launch_bounds__(256) k_sigma_sym_gather(const Item* __restrict__ items,
                                                          const Work* __restrict__ work,
                                                          const double* __restrict__ Garena,
                                                          double* __restrict__ Sarena,
                                                          int64_t ntot,
                                                          const DavState* __restrict__ st,
                                                          int slot) {
  __shared__ int8_t cls_of[kMaxPair];
  __shared__ int32_t cls0[kIrreps + 1];
  __shared__ int32_t nbc[kIrreps];
  __shared__ int64_t gofs[kIrreps][kIrreps];
  const Work wk = work[blockIdx.x];
  const Item& I = items[wk.item];
  const DavState& S = st[wk.item];
  if (!item_active(S, slot)) return;  // uniform over the block (one item)
  const SymInfo& Y = *I.sym;
  const int t = threadIdx.x;
  for (int j = t; j < Y.npair; j += 256) cls_of[j] = Y.cls_of[j];
  if (t <= kIrreps) cls0[t] = Y.cls0[t];
  if (t < kIrreps) nbc[t] = Y.nbc[t];
  if (t < kIrreps * kIrreps) gofs[t >> 3][t & 7] = Y.gofs[t >> 3][t & 7];
  __syncthreads();
  const int64_t K = (int64_t)wk.begin * blockDim.x + t;
  if (K >= I.ndet) return;
  const int vs = vec_slot(S, slot);
  const int G = Y.wfn;
  int a = 0;
  while (a < kIrreps - 1 && K >= Y.blk[a + 1]) ++a;
  const int b = a ^ G;
  const int64_t loc = K - Y.blk[a];
  const int ia = (int)(loc / nbc[b]), ib = (int)(loc % nbc[b]);
  const double* __restrict__ Gi = Garena + I.goff;
  double acc0 = 0.0, acc1 = 0.0;
  const uint32_t* __restrict__ la = I.linkA + (int64_t)(Y.na0[a] + ia) * I.La;
  for (int l = 0; l < I.La; ++l) {
    const uint32_t e = ldg(la + l);
    const int j = link_pair(e), s = cls_of[j];
    const int c0 = cls0[s], nps = cls0[s + 1] - c0;
    acc0 += link_sign(e) * ldg(Gi + gofs[s][a ^ s] +
                               ((int64_t)link_addr(e) * nps + (j - c0)) * nbc[b] + ib);
  }
  const uint32_t* __restrict__ lb = I.linkBT + Y.nb0[b] + ib;  // link l: lb[l * Nb]
  for (int l = 0; l < I.Lb; ++l) {
    const uint32_t e = ldg(lb + (int64_t)l * I.Nb);
    const int j = link_pair(e), s = cls_of[j];
    const int c0 = cls0[s], nps = cls0[s + 1] - c0;
    acc1 += link_sign(e) * ldg(Gi + gofs[s][a] +
                               ((int64_t)ia * nps + (j - c0)) * nbc[b ^ s] + link_addr(e));
  }
  Sarena[(int64_t)vs * ntot + I.off + K] = acc0 + acc1;
}

// ---------------------------------------------------------------- Davidson
// Block-level fixed-order reduction of NV values per thread (256 threads).
template <int NV>
__device__ inline void block_reduce_store(double (&v)[NV], double* out) {
  __shared__ double red[4][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double x = v[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if (lane == 0) red[wave][i] = x;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NV; i += blockDim.x)
    out[i] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
  __syncthreads();
}

constexpr int kPart = kMaxSpace + 2;  // partial sums per chunk
constexpr int kChunk = 4096;          // elements per reduction chunk

// zero a vector slot range for the given items (fill kernel; graph safe)
__global__ void k_fill(double* p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Dense guess vector: r_K = +-1/sqrt(ndet) with the sign taken from the top
// bit of a multiplicative hash of the address K.  It has no symmetry, so it
// carries weight in every spin and spatial symmetry sector of the
// determinant basis: with it in the first subspace the solver cannot be
// confined to a sector without the ground state (a closed-shell determinant,
// for example, is a pure singlet and never reaches a triplet ground state).
__device__ inline double hash_sign(int64_t K) {
  return (((uint64_t)K * 0x9E3779B97F4A7C15ull) >> 63) ? 1.0 : -1.0;
}

// Guess: the `nguess` lowest diagonal determinants (ties: lower address) as
// unit vectors in slots 0..g-1, and the dense vector orthogonalised against
// them in slot g.  One block per item.
__global__ void k_dav_guess(const Item* __restrict__ items, int ibase,
                            const double* __restrict__ diag, double* V, int64_t ntot, DavState* st,
                            int nguess) {
  const Item& I = items[ibase + blockIdx.x];
  DavState& S = st[ibase + blockIdx.x];
  const int t = threadIdx.x;
  constexpr int G = 8;
  double bv[G];
  int64_t bi[G];
  for (int g = 0; g < G; ++g) { bv[g] = 1e300; bi[g] = INT64_MAX; }
  const double* d = diag + I.off;
  for (int64_t K = t; K < I.ndet; K += blockDim.x) {
    double x = d[K];
    // insert (x, K) into the sorted list (value, then index)
    if (x < bv[G - 1] || (x == bv[G - 1] && K < bi[G - 1])) {
      int p = G - 1;
      while (p > 0 && (x < bv[p - 1] || (x == bv[p - 1] && K < bi[p - 1]))) {
        bv[p] = bv[p - 1]; bi[p] = bi[p - 1]; --p;
      }
      bv[p] = x; bi[p] = K;
    }
  }
  // g rounds of a block-wide argmin over the heads of the per-thread lists
  __shared__ double rv[256];
  __shared__ int64_t ri[256];
  __shared__ int rth[256];
  int g = nguess < G ? nguess : G;
  if (g > I.ndet) g = (int)I.ndet;
  __shared__ int64_t chosen[G];
  int head = 0;
  for (int k = 0; k < g; ++k) {
    rv[t] = head < G ? bv[head] : 1e300;
    ri[t] = head < G ? bi[head] : INT64_MAX;
    rth[t] = t;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w) {
        const double v2 = rv[t + w];
        const int64_t i2 = ri[t + w];
        if (v2 < rv[t] || (v2 == rv[t] && i2 < ri[t])) {
          rv[t] = v2;
          ri[t] = i2;
          rth[t] = rth[t + w];
        }
      }
      __syncthreads();
    }
    if (t == rth[0]) ++head;
    if (t == 0) {
      V[(int64_t)k * ntot + I.off + ri[0]] = 1.0;
      chosen[k] = ri[0];
    }
    __syncthreads();
  }
  // dense vector minus its components on the chosen unit vectors
  const bool dense = I.ndet > g;
  if (dense) {
    const double sc = 1.0 / sqrt((double)(I.ndet - g));
    double* __restrict__ vr = V + (int64_t)g * ntot + I.off;
    for (int64_t K = t; K < I.ndet; K += blockDim.x) {
      bool hit = false;
      for (int j = 0; j < g; ++j) hit |= chosen[j] == K;
      vr[K] = hit ? 0.0 : hash_sign(K) * sc;
    }
  }
  if (t == 0) {
    S.m = 0;
    S.nguess = g + (dense ? 1 : 0);
    S.np = 0;
    S.onepass = 0;
    S.olsen = 0;
    S.iters = 0;
    S.status = 0;
    S.rnorm = 0.0;
    S.conv = 0;
    S.theta = 0.0;
    if (I.ndet == 1) {
      S.conv = 1;
      S.m = 1;
      S.theta = d[0];
    }
  }
}

// partial dots p_i = V_i . S_j over one chunk, for i < m (j = newest or `slot`)
__global__ void __launch_bounds__(256) k_dav_dots(const Item* __restrict__ items,
                                                  const Work* __restrict__ work,
                                                  const double* __restrict__ V,
                                                  const double* __restrict__ Sv, int64_t ntot,
                                                  const DavState* __restrict__ st, int slot,
                                                  double* part) {
  const Work wk = work[blockIdx.x];
  const Item& I = items[wk.item];
  const DavState& S = st[wk.item];
  if (!item_active(S, slot)) return;
  const int j = slot >= 0 ? slot : S.m - 1;
  const int m = j + 1;
  double acc[kMaxSpace];
#pragma unroll
  for (int i = 0; i < kMaxSpace; ++i) acc[i] = 0.0;
  const int64_t e0 = (int64_t)(wk.begin - I.chunk0) * kChunk;
  const int64_t e1 = min(e0 + kChunk, I.ndet);
  const double* sj = Sv + (int64_t)j * ntot + I.off;
  const bool unrolled = with_space(m, [&](auto mc) {
    constexpr int M = decltype(mc)::value;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
      const double s = sj[e];
#pragma unroll
      for (int i = 0; i < M; ++i) acc[i] += V[(int64_t)i * ntot + I.off + e] * s;
    }
  });
  if (!unrolled) {
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
      const double s = sj[e];
  #pragma unroll
      for (int i = 0; i < kMaxSpace; ++i)
        if (i < m) acc[i] += V[(int64_t)i * ntot + I.off + e] * s;
    }
  }
  block_reduce_store<kMaxSpace>(acc, part + (int64_t)wk.begin * kPart);
}

// Symmetric Jacobi eigen-solve of the m x m subspace matrix by one wave of
// 64 lanes, parallel ordering: every round applies m/2 disjoint plane
// rotations at once (round-robin pairing of the indices), m-1 rounds per
// sweep.  A rotation is skipped when |a_pq| <= 1e-18 (|a_pp| + |a_qq|); the
// sweeps stop when a whole sweep rotates nothing.  Returns the lowest
// eigenvalue and its eigenvector (ties: lowest index).
__device__ void wave_jacobi_lowest(double* A, double* B, double* Vm, double* Vt, int m,
                                   double* theta, double* y) {
  const int lane = threadIdx.x & 63;
  __shared__ double rc[kMaxSpace], rt[kMaxSpace];
  __shared__ int partner[kMaxSpace];
  __shared__ int rotated;
  const int N = m + (m & 1);  // even number of players (index m is a dummy when m is odd)
  for (int k = lane; k < m * m; k += 64) Vm[k] = (k / m == k % m) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 40 && N > 1; ++sweep) {
    if (lane == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < N - 1; ++r) {
      // round-robin pairs: position 0 holds index 0, positions 1..N-1 rotate
      if (lane < N / 2) {
        const int k = lane;
        const int a0 = (k == 0) ? 0 : 1 + ((k - 1 + r) % (N - 1));
        const int b0 = 1 + ((N - 2 - k + r) % (N - 1));
        const int p = a0 < b0 ? a0 : b0, q = a0 < b0 ? b0 : a0;
        double c = 1.0, t = 0.0;
        bool rot = false;
        if (q < m) {
          const double apq = A[p * m + q], app = A[p * m + p], aqq = A[q * m + q];
          if (fabs(apq) > 1e-18 * (fabs(app) + fabs(aqq)) && apq != 0.0) {
            const double th = (aqq - app) / (2.0 * apq);
            const double tt = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            t = tt * c;
            rot = true;
          }
        }
        if (p < m) { partner[p] = rot ? q : p; rc[p] = c; rt[p] = rot ? -t : 0.0; }
        if (q < m) { partner[q] = rot ? p : q; rc[q] = c; rt[q] = rot ? t : 0.0; }
        if (rot) rotated = 1;
      }
      __syncthreads();
      // B = A J, V = V J : column j <- c_j col_j + t_j col_partner(j)
      for (int e = lane; e < m * m; e += 64) {
        const int i = e / m, j = e % m, pj = partner[j];
        B[e] = rc[j] * A[i * m + j] + rt[j] * A[i * m + pj];
        Vt[e] = rc[j] * Vm[i * m + j] + rt[j] * Vm[i * m + pj];
      }
      __syncthreads();
      // A = J^T B : row i <- c_i row_i + t_i row_partner(i)
      for (int e = lane; e < m * m; e += 64) {
        const int i = e / m, j = e % m, pi = partner[i];
        A[e] = rc[i] * B[i * m + j] + rt[i] * B[pi * m + j];
        Vm[e] = Vt[e];
      }
      __syncthreads();
    }
    if (!rotated) break;
  }
  int best = 0;
  for (int k = 1; k < m; ++k)
    if (A[k * m + k] < A[best * m + best]) best = k;
  *theta = A[best * m + best];
  for (int k = lane; k < m; k += 64) y[k] = Vm[k * m + best];
  __syncthreads();
}

// Reduce the dots of the newest column into Hs; when the subspace is
// complete (guess phase) or always (iteration phase), Rayleigh-Ritz.
// One 64-thread block per item.
__global__ void k_dav_rr(const Item* __restrict__ items, int ibase,
                         const double* __restrict__ part, DavState* st, int slot) {
  const Item& I = items[ibase + blockIdx.x];
  DavState& S = st[ibase + blockIdx.x];
  if (!item_active(S, slot)) return;
  const int j = slot >= 0 ? slot : S.m - 1;
  const int m = j + 1;
  const int lane = threadIdx.x;
  // the Ritz coefficients of the subspace before the newest vector
  const double yold = (lane < kMaxSpace && lane < j) ? S.y[lane] : 0.0;
  if (lane < m) {
    double v = 0.0;
    for (int c = 0; c < I.nchunk; ++c) v += part[(int64_t)(I.chunk0 + c) * kPart + lane];
    S.Hs[lane * kMaxSpace + j] = v;
    S.Hs[j * kMaxSpace + lane] = v;
  }
  __syncthreads();
  const bool solve = slot < 0 || slot == S.nguess - 1;
  if (!solve) return;
  __shared__ double A[kMaxSpace * kMaxSpace], B[kMaxSpace * kMaxSpace];
  __shared__ double Vm[kMaxSpace * kMaxSpace], Vt[kMaxSpace * kMaxSpace], y[kMaxSpace];
  __shared__ double th;
  for (int k = lane; k < m * m; k += 64) A[k] = S.Hs[(k / m) * kMaxSpace + (k % m)];
  __syncthreads();
  double thl;
  wave_jacobi_lowest(A, B, Vm, Vt, m, &thl, y);
  if (lane == 0) th = thl;
  __syncthreads();
  __syncthreads();
  if (lane < kMaxSpace) {
    S.y[lane] = lane < m ? y[lane] : 0.0;
    S.yp[lane] = yold;
  }
  if (lane == 0) {
    S.theta = th;
    if (slot >= 0) {   // end of the guess phase
      S.m = m;
    } else {
      S.iters += 1;
    }
  }
}

// Restart: when the subspace is full, collapse it onto the Ritz vector
// x = V y (and H x = S y) in slot 0 and the previous iteration's Ritz vector,
// made orthogonal to x, in slot 1: z = yp - (y.yp) y in the subspace's
// orthonormal basis, x' = V z / |z| (kept when |z| > kRestartMin).  The
// projected matrix becomes diag(theta, z^T Hs z / |z|^2): y is an
// eigenvector of Hs and z is orthogonal to it.
// Both collapse kernels call restart_coef and must take the same decision:
// explicit fused multiply-adds fix its rounding wherever it is inlined.
constexpr double kRestartMin = 1e-8;
__device__ inline double restart_coef(const DavState& S, double* z) {
  double c = 0.0;
  for (int i = 0; i < S.m; ++i) c = fma(S.y[i], S.yp[i], c);
  double nz = 0.0;
  for (int i = 0; i < S.m; ++i) {
    z[i] = fma(-c, S.y[i], S.yp[i]);
    nz = fma(z[i], z[i], nz);
  }
  nz = sqrt(nz);
  return nz > kRestartMin ? nz : 0.0;
}
__global__ void __launch_bounds__(256) k_dav_collapse(const Item* __restrict__ items,
                                                      const Work* __restrict__ work, double* V,
                                                      double* Sv, int64_t ntot,
                                                      const DavState* __restrict__ st, int mmax) {
  const Work wk = work[blockIdx.x];
  const Item& I = items[wk.item];
  const DavState& S = st[wk.item];
  if (S.conv || S.m < mmax) return;
  __shared__ double z[kMaxSpace];
  __shared__ double nz;
  if (threadIdx.x == 0) nz = restart_coef(S, z);
  __syncthreads();
  const double inv = nz > 0.0 ? 1.0 / nz : 0.0;
  const int64_t e0 = (int64_t)(wk.begin - I.chunk0) * kChunk;
  const int64_t e1 = min(e0 + kChunk, I.ndet);
  const bool unrolled = with_space(S.m, [&](auto mc) {
    constexpr int M = decltype(mc)::value;
    double y[M > 0 ? M : 1], zz[M > 0 ? M : 1];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      y[i] = S.y[i];
      zz[i] = z[i];
    }
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
      double x = 0.0, sx = 0.0, xp = 0.0, sxp = 0.0;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const double v = V[(int64_t)i * ntot + I.off + e];
        const double s = Sv[(int64_t)i * ntot + I.off + e];
        x += y[i] * v;
        sx += y[i] * s;
        xp += zz[i] * v;
        sxp += zz[i] * s;
      }
      V[I.off + e] = x;
      Sv[I.off + e] = sx;
      if (nz > 0.0) {
        V[ntot + I.off + e] = xp * inv;
        Sv[ntot + I.off + e] = sxp * inv;
      }
    }
  });
  if (!unrolled) {
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
      double x = 0.0, sx = 0.0, xp = 0.0, sxp = 0.0;
      for (int i = 0; i < S.m; ++i) {
        const double v = V[(int64_t)i * ntot + I.off + e];
        const double s = Sv[(int64_t)i * ntot + I.off + e];
        x += S.y[i] * v;
        sx += S.y[i] * s;
        xp += z[i] * v;
        sxp += z[i] * s;
      }
      V[I.off + e] = x;
      Sv[I.off + e] = sx;
      if (nz > 0.0) {
        V[ntot + I.off + e] = xp * inv;
        Sv[ntot + I.off + e] = sxp * inv;
      }
    }
  }
}
__global__ void k_dav_collapse_state(const Item* __restrict__ items, DavState* st, int ibase,
                                     int nitem, int mmax) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nitem) return;
  i += ibase;
  DavState& S = st[i];
  if (S.conv || S.m < mmax) return;
  double z[kMaxSpace];
  const double nz = restart_coef(S, z);
  double h11 = 0.0;
  if (nz > 0.0) {
    for (int a = 0; a < S.m; ++a) {
      double row = 0.0;
      for (int b = 0; b < S.m; ++b) row += S.Hs[a * kMaxSpace + b] * z[b];
      h11 += z[a] * row;
    }
    h11 /= nz * nz;
  }
  S.Hs[0] = S.theta;
  S.Hs[1] = 0.0;
  S.Hs[kMaxSpace] = 0.0;
  S.Hs[kMaxSpace + 1] = h11;
  S.m = nz > 0.0 ? 2 : 1;
  S.y[0] = 1.0;
  for (int k = 1; k < kMaxSpace; ++k) S.y[k] = 0.0;
}

// Residual r = S y - theta V y, preconditioned t = r / (theta - H_II) into
// slot m; partial sums of V_i . t (i < m), |r|^2 (index kMaxSpace) and |t|^2
// (index kMaxSpace + 1).
__global__ void __launch_bounds__(256) k_dav_residual(const Item* __restrict__ items,
                                                      const Work* __restrict__ work, double* V,
                                                      const double* __restrict__ Sv,
                                                      const double* __restrict__ diag,
                                                      int64_t ntot,
                                                      const DavState* __restrict__ st,
                                                      double* part) {
  const Work wk = work[blockIdx.x];
  const Item& I = items[wk.item];
  const DavState& S = st[wk.item];
  if (S.conv || S.olsen) return;
  const int m = S.m;
  const double th = S.theta;
  double y[kMaxSpace];
#pragma unroll
  for (int i = 0; i < kMaxSpace; ++i) y[i] = S.y[i];
  double acc[kMaxSpace + 2];
#pragma unroll
  for (int i = 0; i <= kMaxSpace + 1; ++i) acc[i] = 0.0;
  const int64_t e0 = (int64_t)(wk.begin - I.chunk0) * kChunk;
  const int64_t e1 = min(e0 + kChunk, I.ndet);
  double* t_out = V + (int64_t)m * ntot + I.off;
  const bool unrolled = with_space(m, [&](auto mc) {
    constexpr int M = decltype(mc)::value;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
      double r = 0.0;
      double v[M > 0 ? M : 1];
#pragma unroll
      for (int i = 0; i < M; ++i) {
        v[i] = V[(int64_t)i * ntot + I.off + e];
        r += y[i] * (Sv[(int64_t)i * ntot + I.off + e] - th * v[i]);
      }
      acc[kMaxSpace] += r * r;
      double den = th - diag[I.off + e];
      if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
      const double tv = r / den;
      t_out[e] = tv;
      acc[kMaxSpace + 1] += tv * tv;
#pragma unroll
      for (int i = 0; i < M; ++i) acc[i] += v[i] * tv;
    }
  });
  if (!unrolled) {
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
      double r = 0.0;
      double v[kMaxSpace];
  #pragma unroll
      for (int i = 0; i < kMaxSpace; ++i) {
        v[i] = 0.0;
        if (i < m) {
          v[i] = V[(int64_t)i * ntot + I.off + e];
          r += y[i] * (Sv[(int64_t)i * ntot + I.off + e] - th * v[i]);
        }
      }
      acc[kMaxSpace] += r * r;
      double den = th - diag[I.off + e];
      if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
      const double tv = r / den;
      t_out[e] = tv;
      acc[kMaxSpace + 1] += tv * tv;
  #pragma unroll
      for (int i = 0; i < kMaxSpace; ++i)
        if (i < m) acc[i] += v[i] * tv;
    }
  }
  block_reduce_store<kMaxSpace + 2>(acc, part + (int64_t)wk.begin * kPart);
}

// Olsen-corrected preconditioner.  With x = V y the Ritz vector and
// r = S y - theta x its residual, the correction is
//   t = -(D - theta)^{-1} (r - eps x),  eps = x^T (D-theta)^{-1} r / x^T (D-theta)^{-1} x,
// the choice that makes t orthogonal to x (Olsen, Jorgensen and Simons'
// correction of the diagonal-preconditioned update used in FCI codes).
// Pass 1 stores r and x and reduces |r|^2, x.(D-theta)^{-1} r, x.(D-theta)^{-1} x.
__device__ inline double guarded_den(double d) {
  return fabs(d) < 1e-8 ? (d < 0 ? -1e-8 : 1e-8) : d;
}

__global__ void __launch_bounds__(256) k_dav_residual_olsen(
    const Item* __restrict__ items, const Work* __restrict__ work, const double* __restrict__ V,
    const double* __restrict__ Sv, const double* __restrict__ diag, int64_t ntot,
    const DavState* __restrict__ st, double* __restrict__ Rb, double* __restrict__ Xb,
    double* part, int all) {
  const Work wk = work[blockIdx.x];
  const Item& I = items[wk.item];
  const DavState& S = st[wk.item];
  if (S.conv || !(all || S.olsen)) return;
  const int m = S.m;
  const double th = S.theta;
  double y[kMaxSpace];
#pragma unroll
  for (int i = 0; i < kMaxSpace; ++i) y[i] = S.y[i];
  double acc[3] = {0.0, 0.0, 0.0};
  const int64_t e0 = (int64_t)(wk.begin - I.chunk0) * kChunk;
  const int64_t e1 = min(e0 + kChunk, I.ndet);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    double x = 0.0, sx = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxSpace; ++i)
      if (i < m) {
        x += y[i] * V[(int64_t)i * ntot + I.off + e];
        sx += y[i] * Sv[(int64_t)i * ntot + I.off + e];
      }
    const double r = sx - th * x;
    const double den = guarded_den(diag[I.off + e] - th);
    Rb[I.off + e] = r;
    Xb[I.off + e] = x;
    acc[0] += r * r;
    acc[1] += x * r / den;
    acc[2] += x * x / den;
  }
  block_reduce_store<3>(acc, part + (int64_t)wk.begin * kPart);
}

__global__ void k_dav_reduce1_olsen(const Item* __restrict__ items,
                                    const double* __restrict__ part, DavState* st, int ibase,
                                    int nitem, double tol, int max_iter, int all) {
  int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= nitem) return;
  it += ibase;
  const Item& I = items[it];
  DavState& S = st[it];
  if (S.conv || !(all || S.olsen)) return;
  double rr = 0.0, a = 0.0, b = 0.0;
  for (int c = 0; c < I.nchunk; ++c) {
    const double* p = part + (int64_t)(I.chunk0 + c) * kPart;
    rr += p[0];
    a += p[1];
    b += p[2];
  }
  S.rnorm = sqrt(rr);
  S.eps = (b != 0.0) ? a / b : 0.0;
  if (S.rnorm <= tol || S.m >= I.ndet) {
    S.conv = 1;
  } else if (S.iters >= max_iter) {
    S.conv = 1;
    S.status = 1;
  }
}

// t = -(r - eps x) / (D - theta) into slot m; partial dots V_i . t (i < m)
__global__ void __launch_bounds__(256) k_dav_precond_olsen(
    const Item* __restrict__ items, const Work* __restrict__ work, double* V,
    const double* __restrict__ diag, int64_t ntot, const DavState* __restrict__ st,
    const double* __restrict__ Rb, const double* __restrict__ Xb, double* part, int all) {
  const Work wk = work[blockIdx.x];
  const Item& I = items[wk.item];
  const DavState& S = st[wk.item];
  if (S.conv || !(all || S.olsen)) return;
  const int m = S.m;
  const double th = S.theta, eps = S.eps;
  double acc[kMaxSpace];
#pragma unroll
  for (int i = 0; i < kMaxSpace; ++i) acc[i] = 0.0;
  const int64_t e0 = (int64_t)(wk.begin - I.chunk0) * kChunk;
  const int64_t e1 = min(e0 + kChunk, I.ndet);
  double* t_out = V + (int64_t)m * ntot + I.off;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const double den = guarded_den(diag[I.off + e] - th);
    const double tv = -(Rb[I.off + e] - eps * Xb[I.off + e]) / den;
    t_out[e] = tv;
#pragma unroll
    for (int i = 0; i < kMaxSpace; ++i)
      if (i < m) acc[i] += V[(int64_t)i * ntot + I.off + e] * tv;
  }
  block_reduce_store<kMaxSpace>(acc, part + (int64_t)wk.begin * kPart);
}

// first Gram-Schmidt coefficients from the partial dots
__global__ void k_dav_reduce_coef(const Item* __restrict__ items, const double* __restrict__ part,
                                  DavState* st, int ibase, int nitem, int all) {
  int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= nitem) return;
  it += ibase;
  const Item& I = items[it];
  DavState& S = st[it];
  if (S.conv || !(all || S.olsen)) return;
  double cf[kMaxSpace];
  for (int i = 0; i < kMaxSpace; ++i) cf[i] = 0.0;
  for (int c = 0; c < I.nchunk; ++c) {
    const double* p = part + (int64_t)(I.chunk0 + c) * kPart;
    for (int i = 0; i < S.m; ++i) cf[i] += p[i];
  }
  for (int i = 0; i < kMaxSpace; ++i) S.coef[i] = cf[i];
  S.onepass = 0;
}

// Convergence test and first Gram-Schmidt coefficients.  An unconverged
// item whose residual fell below olsen_below takes the Olsen correction from
// the next iteration on (0: never).
__global__ void k_dav_reduce1(const Item* __restrict__ items, const double* __restrict__ part,
                              const double* __restrict__ pdots, DavState* st, int ibase,
                              int nitem, double tol, int max_iter, double olsen_below) {
  int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= nitem) return;
  it += ibase;
  const Item& I = items[it];
  DavState& S = st[it];
  if (S.conv || S.olsen) return;
  double rr = 0.0, tt = 0.0;
  double cf[kMaxSpace];
  for (int i = 0; i < kMaxSpace; ++i) cf[i] = 0.0;
  for (int c = 0; c < I.nchunk; ++c) {
    const double* p = part + (int64_t)(I.chunk0 + c) * kPart;
    rr += p[kMaxSpace];
    tt += p[kMaxSpace + 1];
    for (int i = 0; i < S.m; ++i) cf[i] += p[i];
  }
  if (pdots && S.np > 0) {  // the P-space correction changed t on the P block
    const double* pd = pdots + (int64_t)it * (kMaxSpace + 1);
    for (int i = 0; i < S.m; ++i) cf[i] += pd[i];
    tt += pd[kMaxSpace];
  }
  S.rnorm = sqrt(rr);
  for (int i = 0; i < kMaxSpace; ++i) S.coef[i] = cf[i];
  // one Gram-Schmidt pass suffices when it keeps at least half of |t|^2
  // (the Daniel-Gragg-Kaufman-Stewart criterion); |t - V c|^2 = |t|^2 - |c|^2
  double n1 = tt;
  for (int i = 0; i < S.m; ++i) n1 -= cf[i] * cf[i];
  S.onepass = (n1 >= 0.5 * tt && n1 > 1e-28) ? 1 : 0;
  S.tnorm2 = n1;
  if (S.rnorm <= tol || S.m >= I.ndet) {
    S.conv = 1;
  } else if (S.iters >= max_iter) {
    S.conv = 1;
    S.status = 1;
  } else if (S.rnorm < olsen_below) {
    S.olsen = 1;
  }
}

// t -= sum_i coef_i V_i ; partial sums of V_i . t and |t|^2 (second pass).
// Items whose first pass suffices (onepass) are normalised here instead.
__global__ void __launch_bounds__(256) k_dav_orth(const Item* __restrict__ items,
                                                  const Work* __restrict__ work, double* V,
                                                  int64_t ntot, const DavState* __restrict__ st,
                                                  double* part) {
  const Work wk = work[blockIdx.x];
  const Item& I = items[wk.item];
  const DavState& S = st[wk.item];
  if (S.conv) return;
  const int m = S.m;
  double cf[kMaxSpace];
#pragma unroll
  for (int i = 0; i < kMaxSpace; ++i) cf[i] = S.coef[i];
  if (S.onepass) {
    const double inv = 1.0 / sqrt(S.tnorm2);
    const int64_t e0 = (int64_t)(wk.begin - I.chunk0) * kChunk;
    const int64_t e1 = min(e0 + kChunk, I.ndet);
    double* t = V + (int64_t)m * ntot + I.off;
    const bool unrolled = with_space(m, [&](auto mc) {
      constexpr int M = decltype(mc)::value;
      for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
        double tv = t[e];
#pragma unroll
        for (int i = 0; i < M; ++i) tv -= cf[i] * V[(int64_t)i * ntot + I.off + e];
        t[e] = tv * inv;
      }
    });
    if (!unrolled) {
      for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
        double tv = t[e];
  #pragma unroll
        for (int i = 0; i < kMaxSpace; ++i)
          if (i < m) tv -= cf[i] * V[(int64_t)i * ntot + I.off + e];
        t[e] = tv * inv;
      }
    }
    return;
  }
  double acc[kMaxSpace + 1];
#pragma unroll
  for (int i = 0; i <= kMaxSpace; ++i) acc[i] = 0.0;
  const int64_t e0 = (int64_t)(wk.begin - I.chunk0) * kChunk;
  const int64_t e1 = min(e0 + kChunk, I.ndet);
  double* t = V + (int64_t)m * ntot + I.off;
  const bool unrolled = with_space(m, [&](auto mc) {
    constexpr int M = decltype(mc)::value;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
      double v[M > 0 ? M : 1];
      double tv = t[e];
#pragma unroll
      for (int i = 0; i < M; ++i) {
        v[i] = V[(int64_t)i * ntot + I.off + e];
        tv -= cf[i] * v[i];
      }
      t[e] = tv;
#pragma unroll
      for (int i = 0; i < M; ++i) acc[i] += v[i] * tv;
      acc[kMaxSpace] += tv * tv;
    }
  });
  if (!unrolled) {
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
      double v[kMaxSpace];
      double tv = t[e];
  #pragma unroll
      for (int i = 0; i < kMaxSpace; ++i) {
        v[i] = 0.0;
        if (i < m) {
          v[i] = V[(int64_t)i * ntot + I.off + e];
          tv -= cf[i] * v[i];
        }
      }
      t[e] = tv;
  #pragma unroll
      for (int i = 0; i < kMaxSpace; ++i)
        if (i < m) acc[i] += v[i] * tv;
      acc[kMaxSpace] += tv * tv;
    }
  }
  block_reduce_store<kMaxSpace + 1>(acc, part + (int64_t)wk.begin * kPart);
}

__global__ void k_dav_reduce2(const Item* __restrict__ items, const double* __restrict__ part,
                              DavState* st, int ibase, int nitem) {
  int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= nitem) return;
  it += ibase;
  const Item& I = items[it];
  DavState& S = st[it];
  if (S.conv || S.onepass) return;
  double tt = 0.0;
  double cf[kMaxSpace];
  for (int i = 0; i < kMaxSpace; ++i) cf[i] = 0.0;
  for (int c = 0; c < I.nchunk; ++c) {
    const double* p = part + (int64_t)(I.chunk0 + c) * kPart;
    tt += p[kMaxSpace];
    for (int i = 0; i < S.m; ++i) cf[i] += p[i];
  }
  double n2 = tt;
  for (int i = 0; i < S.m; ++i) n2 -= cf[i] * cf[i];
  for (int i = 0; i < kMaxSpace; ++i) S.coef[i] = cf[i];
  S.tnorm2 = n2;
  if (!(n2 > 1e-28)) {  // the correction lies in the subspace: accept
    S.conv = 1;
    S.status = 2;
  }
}

// t -= sum_i coef_i V_i, t /= |t|: the new basis vector in slot m; m += 1.
__global__ void __launch_bounds__(256) k_dav_orth2(const Item* __restrict__ items,
                                                   const Work* __restrict__ work, double* V,
                                                   int64_t ntot, const DavState* __restrict__ st) {
  const Work wk = work[blockIdx.x];
  const Item& I = items[wk.item];
  const DavState& S = st[wk.item];
  if (S.conv || S.onepass) return;
  const int m = S.m;
  double cf[kMaxSpace];
#pragma unroll
  for (int i = 0; i < kMaxSpace; ++i) cf[i] = S.coef[i];
  const double inv = 1.0 / sqrt(S.tnorm2);
  const int64_t e0 = (int64_t)(wk.begin - I.chunk0) * kChunk;
  const int64_t e1 = min(e0 + kChunk, I.ndet);
  double* t = V + (int64_t)m * ntot + I.off;
  const bool unrolled = with_space(m, [&](auto mc) {
    constexpr int M = decltype(mc)::value;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
      double tv = t[e];
#pragma unroll
      for (int i = 0; i < M; ++i) tv -= cf[i] * V[(int64_t)i * ntot + I.off + e];
      t[e] = tv * inv;
    }
  });
  if (!unrolled) {
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
      double tv = t[e];
  #pragma unroll
      for (int i = 0; i < kMaxSpace; ++i)
        if (i < m) tv -= cf[i] * V[(int64_t)i * ntot + I.off + e];
      t[e] = tv * inv;
    }
  }
}
__global__ void k_dav_grow(DavState* st, int ibase, int nitem) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nitem) return;
  i += ibase;
  DavState& S = st[i];
  if (!S.conv) S.m += 1;
}

// ------------------------------------------------------------- P-space
// Davidson with a P-space: the np = min(kMaxPspace-ish cap, ndet) determinants
// of lowest diagonal energy (ties: lower address) span a block H_PP of H that
// is diagonalised exactly once per CASCI, H_PP = U diag(lambda) U^T.  It
// supplies (i) the guess, the lowest eigenvector of H_PP plus the
// lowest-diagonal unit vector orthogonalised against it (so every spin and
// spatial symmetry sector of the determinant basis stays in the subspace),
// and (ii) the preconditioner: the correction t = (theta - H)^-1 r is
// approximated by (theta - H_PP)^-1 r on the P block and by the diagonal
// (theta - H_II)^-1 r elsewhere.  The converged eigenpair does not depend on
// either choice, only the number of iterations does.

// Orderable 64-bit key of a double (ascending unsigned order = ascending
// value; -0 and +0 share the key of +0).
__device__ inline uint64_t order_key(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x == 0.0 ? 0.0 : x);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// The np lowest of n distinct 96-bit keys (key_at(i) -> order_key(H_II) and
// address) by radix select in 8-bit digits (12 histogram passes: 8 over the
// value key from the top, 4 over the address), then every key up to the np-th
// is collected, unordered, into khi/klo (exactly min(np, n) of them).
// 256 threads.
template <class KeyAt>
__device__ void select_lowest(const KeyAt& key_at, int64_t n, int np, uint64_t* khi,
                              uint32_t* klo) {
  const int t = threadIdx.x;
  __shared__ uint32_t hist[256];
  __shared__ uint64_t pre_hi;
  __shared__ uint32_t pre_lo;
  __shared__ int64_t need;
  __shared__ uint32_t ncol;
  if (t == 0) { pre_hi = 0; pre_lo = 0; need = np; ncol = 0; }
  __syncthreads();
  if (np < n) {
    for (int dg = 0; dg < 12; ++dg) {
      hist[t] = 0;
      __syncthreads();
      const uint64_t ph = pre_hi;
      const uint32_t pl = pre_lo;
      for (int64_t K = t; K < n; K += 256) {
        uint64_t kh;
        uint32_t kl;
        key_at(K, kh, kl);
        bool match;
        int b;
        if (dg < 8) {
          const int sh = 56 - 8 * dg;
          match = dg == 0 || (kh >> (sh + 8)) == (ph >> (sh + 8));
          b = (int)((kh >> sh) & 0xFF);
        } else {
          const int sh = 24 - 8 * (dg - 8);
          match = kh == ph && (dg == 8 || (kl >> (sh + 8)) == (pl >> (sh + 8)));
          b = (int)((kl >> sh) & 0xFF);
        }
        if (match) atomicAdd(&hist[b], 1u);
      }
      __syncthreads();
      if (t == 0) {
        int64_t k = need, cum = 0;
        int b = 0;
        for (; b < 255; ++b) {
          if (cum + hist[b] >= k) break;
          cum += hist[b];
        }
        need = k - cum;
        if (dg < 8) pre_hi |= (uint64_t)b << (56 - 8 * dg);
        else pre_lo |= (uint32_t)b << (24 - 8 * (dg - 8));
      }
      __syncthreads();
    }
  } else if (t == 0) {
    pre_hi = ~0ull;
    pre_lo = ~0u;
  }
  __syncthreads();
  const uint64_t ph = pre_hi;
  const uint32_t pl = pre_lo;
  for (int64_t K = t; K < n; K += 256) {
    uint64_t kh;
    uint32_t kl;
    key_at(K, kh, kl);
    if (kh < ph || (kh == ph && kl <= pl)) {
      const uint32_t slot = atomicAdd(&ncol, 1u);
      if (slot < (uint32_t)kMaxPspace) { khi[slot] = kh; klo[slot] = kl; }
    }
  }
  __syncthreads();
}

// P-space size requested from the selection: every determinant of a small
// CASCI, else pmax (at least the eight lowest, the unit guesses when the
// P-space is not used).
__device__ __forceinline__ int select_count(int64_t nd, int pmax) {
  return nd <= kMaxPspace ? (int)nd : (pmax > 8 ? pmax : 8);
}

// First phase for CASCIs of more than kSelectChunk determinants: one block per
// chunk of kSelectChunk addresses writes the chunk's np lowest keys to the
// item's candidate slots (chunk c of an item whose slots start at s:
// slot s + c, kMaxPspace keys each; unused keys are the sentinel ~0, which is
// never selected since the item has at least np real keys).  Work: item,
// chunk index, first slot of the item.
__global__ void __launch_bounds__(256) k_pspace_select_chunk(const Item* __restrict__ items,
                                                             const Work* __restrict__ work,
                                                             int ibase, int nitem,
                                                             const double* __restrict__ diag,
                                                             uint64_t* __restrict__ cand_hi,
                                                             uint32_t* __restrict__ cand_lo,
                                                             int pmax) {
  const Work wk = work[blockIdx.x];
  if (wk.item < ibase || wk.item >= ibase + nitem) return;
  const Item& I = items[wk.item];
  const int np = select_count(I.ndet, pmax);
  const int64_t lo = (int64_t)wk.begin * kSelectChunk;
  const int64_t hi = min(I.ndet, lo + kSelectChunk);
  const double* __restrict__ d = diag + I.off;
  __shared__ uint64_t khi[kMaxPspace];
  __shared__ uint32_t klo[kMaxPspace];
  auto key_at = [&](int64_t i, uint64_t& kh, uint32_t& kl) {
    kh = order_key(d[lo + i]);
    kl = (uint32_t)(lo + i);
  };
  const int64_t n = hi - lo;
  select_lowest(key_at, n, np, khi, klo);
  const int got = n < np ? (int)n : np;
  const int64_t s = ((int64_t)wk.end + wk.begin) * kMaxPspace;
  for (int j = threadIdx.x; j < kMaxPspace; j += 256) {
    cand_hi[s + j] = j < got ? khi[j] : ~0ull;
    cand_lo[s + j] = j < got ? klo[j] : ~0u;
  }
}

// Selection of the np lowest (diagonal, address) keys of one item, then a rank
// sort of the np survivors; pidx[item][k] receives the addresses in ascending
// key order.  One 256-thread block per item.  An item with candidate slots
// (cand_slot[item] >= 0, filled by k_pspace_select_chunk) selects among them;
// the others read the diagonal directly.
__global__ void __launch_bounds__(256) k_pspace_select(const Item* __restrict__ items, int ibase,
                                                       const double* __restrict__ diag,
                                                       int32_t* __restrict__ pidx, int pmax,
                                                       const int32_t* __restrict__ cand_slot,
                                                       const uint64_t* __restrict__ cand_hi,
                                                       const uint32_t* __restrict__ cand_lo) {
  const int it = ibase + blockIdx.x;
  const Item& I = items[it];
  const int64_t nd = I.ndet;
  const int np = select_count(nd, pmax);
  const int t = threadIdx.x;
  __shared__ uint64_t khi[kMaxPspace];
  __shared__ uint32_t klo[kMaxPspace];
  const int slot = cand_slot ? cand_slot[it] : -1;
  if (slot >= 0) {
    const int64_t nchunk = (nd + kSelectChunk - 1) / kSelectChunk;
    const uint64_t* __restrict__ ch = cand_hi + (int64_t)slot * kMaxPspace;
    const uint32_t* __restrict__ cl = cand_lo + (int64_t)slot * kMaxPspace;
    auto key_at = [&](int64_t i, uint64_t& kh, uint32_t& kl) {
      kh = ch[i];
      kl = cl[i];
    };
    select_lowest(key_at, nchunk * kMaxPspace, np, khi, klo);
  } else {
    const double* __restrict__ d = diag + I.off;
    auto key_at = [&](int64_t i, uint64_t& kh, uint32_t& kl) {
      kh = order_key(d[i]);
      kl = (uint32_t)i;
    };
    select_lowest(key_at, nd, np, khi, klo);
  }
  // rank sort (keys are distinct)
  if (t < np) {
    const uint64_t kh = khi[t];
    const uint32_t kl = klo[t];
    int rank = 0;
    for (int j = 0; j < np; ++j)
      rank += (khi[j] < kh || (khi[j] == kh && klo[j] < kl)) ? 1 : 0;
    pidx[(int64_t)it * kMaxPspace + rank] = (int32_t)kl;
  }
}

// Matrix element <I|H - E_core|J> between two different determinants of the
// active space (Slater-Condon rules; strings are bit masks over the active
// orbitals, alpha string before beta string, each in ascending order).
__device__ inline int between_parity(uint64_t s, int p, int q) {
  const int lo = p < q ? p : q, hi = p < q ? q : p;
  const uint64_t m = (((uint64_t)1 << hi) - 1) & ~((((uint64_t)1 << lo) << 1) - 1);
  return __builtin_popcountll(s & m) & 1;
}
__device__ double sc_offdiag(const ItemHam& H, uint64_t ia, uint64_t ib, uint64_t ja,
                             uint64_t jb) {
  const uint64_t xa = ia ^ ja, xb = ib ^ jb;
  const int da = __builtin_popcountll(xa) >> 1, db = __builtin_popcountll(xb) >> 1;
  if (da + db > 2) return 0.0;
  const double* __restrict__ eri = H.eri;
  const int M = H.M;
  auto g = [&](int p, int q, int r, int s) -> double {
    return ldg(eri + (((int64_t)H.act[p] * M + H.act[q]) * M + H.act[r]) * M + H.act[s]);
  };
  if (da + db == 1) {
    // one excitation q -> p in the string of spin sigma
    const uint64_t is = da ? ia : ib, js = da ? ja : jb, jo = da ? jb : ja;
    const int p = __builtin_ctzll(is & ~js), q = __builtin_ctzll(js & ~is);
    double v = H.heff[p * kMaxActive + q];
    for (uint64_t x = js; x; x &= x - 1) {
      const int r = __builtin_ctzll(x);
      v += g(p, q, r, r) - g(p, r, r, q);   // r = q contributes zero
    }
    for (uint64_t x = jo; x; x &= x - 1) {
      const int r = __builtin_ctzll(x);
      v += g(p, q, r, r);
    }
    return between_parity(js, p, q) ? -v : v;
  }
  if (da == 1 && db == 1) {
    const int p = __builtin_ctzll(ia & ~ja), q = __builtin_ctzll(ja & ~ia);
    const int r = __builtin_ctzll(ib & ~jb), s = __builtin_ctzll(jb & ~ib);
    const double v = g(p, q, r, s);
    return (between_parity(ja, p, q) ^ between_parity(jb, r, s)) ? -v : v;
  }
  // two excitations in one string: holes q1 < q2, particles p1 < p2;
  // I = E_p1q1 E_p2q2 J (up to the sign), element (p1 q1|p2 q2) - (p1 q2|p2 q1)
  const uint64_t is = da ? ia : ib, js = da ? ja : jb;
  uint64_t pp = is & ~js, hh = js & ~is;
  const int p1 = __builtin_ctzll(pp), p2 = 63 - __builtin_clzll(pp);
  const int q1 = __builtin_ctzll(hh), q2 = 63 - __builtin_clzll(hh);
  const uint64_t k = (js & ~((uint64_t)1 << q2)) | ((uint64_t)1 << p2);
  const int par = between_parity(js, p2, q2) ^ between_parity(k, p1, q1);
  const double v = g(p1, q1, p2, q2) - g(p1, q2, p2, q1);
  return par ? -v : v;
}

// One block per item: build H_PP (packed lower triangle in LDS) and reduce
// it to tridiagonal form by Householder reflections, H_PP = Q T Q^T (T:
// diagonal d, off-diagonal e; Q accumulated explicitly for a P-space).
// The lowest eigenvalue of T comes from multisection on Sturm counts (every
// thread evaluates one point per round), its eigenvector from inverse
// iteration; the guess is Q z.  A CASCI of at most kMaxPspace determinants
// is always solved from its whole-space block (the guess is then the exact
// ground state, whatever pmax); larger ones use a P-space of
// min(pmax, ndet / kPspaceRatio) determinants, since the reduction costs
// about P^3 against a Davidson iteration's ndet npair^2; below kPspaceMinDim
// (where small P-spaces can also steer the solver to an excited root) they
// start from `nunit` lowest-diagonal unit vectors with the diagonal
// correction.  The dense vector is always added.  The reduction runs in
// five instantiations over host-built item lists: P-spaces of larger
// CASCIs (512 threads, Q in LDS; sized for 112 and for 76), and CASCIs
// solved from their whole space of at most 36 determinants (one wave),
// 37..100 and 101..112 (256 threads), which need no Q; the sizes let
// several blocks share a CU.

// Solve (theta - T) z = y for symmetric tridiagonal T (diagonal d, off-
// diagonal e) by an LDL^T sweep without pivoting, pivots kept at |p| >= floor
// (1e-8 for the correction, like the diagonal one; a tiny relative floor for
// inverse iteration).  In the Davidson iteration theta never exceeds the
// lowest eigenvalue of T, so theta - T is negative semidefinite and the sweep
// is stable.  z may alias y.
__device__ inline double floored(double p, double floor) {
  return fabs(p) < floor ? (p < 0 ? -floor : floor) : p;
}
__device__ inline void tridiag_shift_solve(const double* d, const double* e, int n, double theta,
                                           const double* y, double* z, double* piv,
                                           double floor) {
  double p = floored(theta - d[0], floor);
  piv[0] = p;
  z[0] = y[0];
  for (int i = 1; i < n; ++i) {
    const double l = -e[i - 1] / p;           // multiplier of the off-diagonal (-e)
    p = floored((theta - d[i]) + l * e[i - 1], floor);
    piv[i] = p;
    z[i] = y[i] - l * z[i - 1];
  }
  z[n - 1] = z[n - 1] / piv[n - 1];
  for (int i = n - 2; i >= 0; --i) z[i] = (z[i] + e[i] * z[i + 1]) / piv[i];
}

__device__ inline int sturm_count(const double* d, const double* e, int n, double x) {
  int cnt = 0;
  double q = d[0] - x;
  if (q == 0.0) q = -1e-300;
  cnt += q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = (d[i] - x) - e[i - 1] * e[i - 1] / q;
    if (q == 0.0) q = -1e-300;
    cnt += q < 0.0;
  }
  return cnt;
}

// Guess of the CASCIs without a P-space, one 256-thread block per item of
// the view (the others return at once): a single determinant is its own
// solution; otherwise unit vectors on the nunit lowest diagonal determinants
// (idx is sorted) and the dense vector without those components in slot
// nunit.
__global__ void __launch_bounds__(256) k_pspace_guess(const Item* __restrict__ items, int ibase,
                                                      const double* __restrict__ diag,
                                                      const int32_t* __restrict__ pidx, double* V,
                                                      int64_t ntot, DavState* st, int pmax,
                                                      int nunit) {
  const int it = ibase + blockIdx.x;
  const Item& I = items[it];
  DavState& S = st[it];
  const int t = threadIdx.x;
  const int64_t nd = I.ndet;
  const int32_t* __restrict__ idx = pidx + (int64_t)it * kMaxPspace;
  if (nd == 1) {  // nothing to solve: the single determinant
    if (t == 0) {
      V[I.off] = 1.0;
      S.m = 1; S.nguess = 1; S.np = 0; S.iters = 0; S.status = 0; S.rnorm = 0.0; S.conv = 1;
      S.onepass = 0;
      S.olsen = 0;
      S.theta = diag[I.off];
    }
    return;
  }
  if (pspace_dim(nd, pmax) != 0) return;
  const int g = nunit;
  const double sc = 1.0 / sqrt((double)(nd - g));
  double* __restrict__ vr = V + (int64_t)g * ntot + I.off;
  for (int64_t K = t; K < nd; K += 256) {
    bool hit = false;
    for (int j = 0; j < g; ++j) hit |= idx[j] == K;
    vr[K] = hit ? 0.0 : hash_sign(K) * sc;
  }
  if (t < g) V[(int64_t)t * ntot + I.off + idx[t]] = 1.0;
  if (t == 0) {
    S.m = 0; S.nguess = g + 1; S.np = 0; S.iters = 0; S.status = 0; S.rnorm = 0.0; S.conv = 0;
    S.onepass = 0;
    S.olsen = 0;
    S.theta = 0.0;
  }
}

// One block of NT threads per item of plist (absolute item indices).  PMAX
// bounds the P-space held in LDS; EXACT: the items whose P-space is their
// whole space (their guess is exact, so Q is not formed).
template <int PMAX, int NT, bool EXACT>
__global__ void __launch_bounds__(NT) k_pspace_eigen(
    const Item* __restrict__ items, const int32_t* __restrict__ plist,
    const ItemHam* __restrict__ hams, const double* __restrict__ diag,
    const int32_t* __restrict__ pidx, double* __restrict__ pQ, double* __restrict__ pT, double* V,
    int64_t ntot, DavState* st, int pmax) {
  static_assert(NT >= PMAX && NT % 64 == 0, "a thread per P row");
  static_assert(EXACT || NT / 4 >= PMAX, "four threads per column when forming Q");
  constexpr int PM = kMaxPspace;  // stride of the per-item arrays in global memory
  __shared__ double A[PMAX * (PMAX + 1) / 2];
  __shared__ uint64_t sa[PMAX], sb[PMAX];
  __shared__ double vv[PMAX], pw[PMAX], dd[PMAX], ee[PMAX], beta[PMAX], zz[PMAX], piv[PMAX];
  __shared__ double lo_hi[2];
  __shared__ int cnt[NT];
  const int it = plist[blockIdx.x];
  const Item& I = items[it];
  DavState& S = st[it];
  const int t = threadIdx.x, lane = t & 63;
  const int64_t nd = I.ndet;
  const int32_t* __restrict__ idx = pidx + (int64_t)it * PM;
  const int n = pspace_dim(nd, pmax);
  // the list holds only this class (checked again: a mismatch would overrun LDS)
  if (nd == 1 || n == 0 || n > PMAX || (nd == n) != EXACT) return;
  const ItemHam& H = hams[I.ham];
  // Q is accumulated in place in the item's output rows (L2-resident):
  // in LDS it would hold the CU to one workgroup
  double* __restrict__ Q = pQ + (int64_t)it * PM * PM;
  for (int k = t; k < n; k += NT) {
    const int e = idx[k];  // an address of this item: 0 <= e < ndet
    uint64_t ma, mb;
    det_strings(I, e, ma, mb);
    sa[k] = ma;
    sb[k] = mb;
  }
  __syncthreads();
  auto L = [](int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; };
  // the packed lower triangle, its elements dealt evenly over the threads
  // (element x is row i, column x - i(i+1)/2)
  for (int x = t; x < n * (n + 1) / 2; x += NT) {
    int i = (int)((sqrt(8.0 * x + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= x) ++i;
    while (i * (i + 1) / 2 > x) --i;
    const int j = x - i * (i + 1) / 2;
    A[x] = (i == j) ? diag[I.off + idx[i]] : sc_offdiag(H, sa[i], sb[i], sa[j], sb[j]);
  }
  __syncthreads();

  // ---- Householder reduction: step k annihilates A[k+2.., k].  The two
  // dot products of a step are formed by every wave for itself (a butterfly
  // over the wave leaves the same value in every lane of every wave), so a
  // step needs three block barriers.
  auto wave_sum = [&](double x) -> double {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
  };
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double sq = 0.0;
    for (int i = lane; i < m; i += 64) {
      const double xi = A[L(k + 1 + i, k)];
      sq += xi * xi;
    }
    const double sig = wave_sum(sq);
    const double x0 = A[L(k + 1, k)];
    const double sg = sqrt(sig);
    const double alpha = x0 >= 0.0 ? -sg : sg;
    const double bt = sig > 0.0 ? 1.0 / (sig - x0 * alpha) : 0.0;
    if (t < m) vv[t] = t == 0 ? x0 - alpha : A[L(k + 1 + t, k)];
    if (t == 0) {
      ee[k] = sig > 0.0 ? alpha : x0;
      beta[k] = bt;
    }
    __syncthreads();
    if (bt != 0.0) {
      // p = beta B v, four threads per row of the trailing block B
      for (int row0 = 0; row0 < m; row0 += NT / 4) {
        const int row = row0 + (t >> 2), part = t & 3;
        double acc = 0.0;
        if (row < m) {
#pragma unroll 4
          for (int j = part; j < m; j += 4) acc += A[L(k + 1 + row, k + 1 + j)] * vv[j];
        }
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        if (row < m && part == 0) pw[row] = bt * acc;
      }
      __syncthreads();
      double pv = 0.0;
      for (int i = lane; i < m; i += 64) pv += pw[i] * vv[i];
      const double Kc = 0.5 * bt * wave_sum(pv);
      // B -= v w^T + w v^T with w = p - K v (lower triangle), rows strided
      // by 64, columns by 8
      for (int i = t >> 3; i < m; i += NT / 8) {
        const double vi = vv[i], wi = pw[i] - Kc * vi;
#pragma unroll 4
        for (int j = t & 7; j <= i; j += 8)
          A[L(k + 1 + i, k + 1 + j)] -= vi * (pw[j] - Kc * vv[j]) + wi * vv[j];
      }
    }
    // keep v in column k below the diagonal (A[k+1+i, k] = v_i)
    if (t < m) A[L(k + 1 + t, k)] = vv[t];
    __syncthreads();
  }
  for (int i = t; i < n; i += NT) {
    dd[i] = A[L(i, i)];
    if (i == n - 2) ee[i] = A[L(n - 1, n - 2)];
  }
  if (t == 0 && n >= 1) ee[n - 1] = 0.0;
  // A CASCI whose P block is its whole space converges on this guess, so it
  // needs no correction and no explicit Q: the guess Q z is formed from the
  // reflectors below.
  // ---- Q = H_0 H_1 ... H_{n-3}, accumulated backwards from the identity
  if constexpr (!EXACT) {
  for (int x = t; x < n * n; x += NT) Q[(x / n) * PM + (x % n)] = (x / n == x % n) ? 1.0 : 0.0;
  __syncthreads();
  for (int k = n - 3; k >= 0; --k) {
    const int m = n - k - 1;
    const double bt = beta[k];
    if (bt == 0.0) continue;  // uniform
    // s_j = sum_i v_i Q[k+1+i][j] for columns j > k (columns <= k are still
    // those of the identity there); four threads per column
    {
      const int col = k + 1 + (t >> 2), part = t & 3;
      double acc = 0.0;
      if (col < n) {
#pragma unroll 4
        for (int i = part; i < m; i += 4) acc += A[L(k + 1 + i, k)] * Q[(k + 1 + i) * PM + col];
      }
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      if (col < n && part == 0) pw[col - k - 1] = bt * acc;
    }
    __syncthreads();
    // element x = i m + j of the trailing block, x = t, t + NT, ... (the
    // row and column step by NT / m and NT % m)
    {
      const int di = NT / m, dj = NT % m;
      int i = t / m, j = t % m;
      while (i < m) {
        Q[(k + 1 + i) * PM + (k + 1 + j)] -= A[L(k + 1 + i, k)] * pw[j];
        i += di;
        j += dj;
        if (j >= m) {
          j -= m;
          ++i;
        }
      }
    }
    __syncthreads();
  }
  }
  // ---- lowest eigenvalue of T: multisection on [lo, hi] (Gershgorin)
  if (t == 0) {
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < n; ++i) {
      const double rr = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < n ? fabs(ee[i]) : 0.0);
      lo = fmin(lo, dd[i] - rr);
      hi = fmax(hi, dd[i] + rr);
    }
    lo_hi[0] = lo;
    lo_hi[1] = hi;
  }
  __syncthreads();
  // rounds of NT points narrow the interval by NT^rounds >= 1.8e16, to the
  // rounding level of the spectrum (512^6, 256^7, 64^9)
  constexpr int kRounds = NT >= 512 ? 6 : NT >= 256 ? 7 : 9;
  for (int round = 0; round < kRounds; ++round) {
    const double lo = lo_hi[0], hi = lo_hi[1];
    const double x = lo + (hi - lo) * (double)(t + 1) / (double)NT;
    const int c = sturm_count(dd, ee, n, x);
    // the first point with at least one eigenvalue below it (the count at
    // the previous point is the previous thread's)
    __syncthreads();
    cnt[t] = c;
    __syncthreads();
    if (c >= 1 && (t == 0 || cnt[t - 1] == 0)) {
      lo_hi[0] = lo + (hi - lo) * (double)t / (double)NT;
      lo_hi[1] = x;
    }
    __syncthreads();
  }
  const double lam0 = 0.5 * (lo_hi[0] + lo_hi[1]);
  // ---- eigenvector of T for lam0: inverse iteration, (lam0 - T) z = z, with
  // pivots floored at 1e-15 of the spectrum's scale
  if (t == 0) {
    double scale = 0.0;
    for (int i = 0; i < n; ++i) scale = fmax(scale, fabs(dd[i]) + 2.0 * fabs(ee[i]));
    const double floor = 1e-15 * fmax(scale, 1e-300);
    for (int i = 0; i < n; ++i) zz[i] = 1.0;
    for (int rep = 0; rep < 3; ++rep) {
      tridiag_shift_solve(dd, ee, n, lam0, zz, zz, piv, floor);
      double s2 = 0.0;
      for (int i = 0; i < n; ++i) s2 += zz[i] * zz[i];
      const double inv = 1.0 / sqrt(s2);
      for (int i = 0; i < n; ++i) zz[i] *= inv;
    }
  }
  __syncthreads();
  // ---- outputs: T and the guess vectors (Q is in place)
  if constexpr (!EXACT) {
    double* __restrict__ To = pT + (int64_t)it * 2 * PM;
    for (int i = t; i < n; i += NT) {
      To[i] = dd[i];
      To[PM + i] = ee[i];
    }
    // u = Q z (row k: P position k)
    if (t < n) {
      double u = 0.0;
      for (int j = 0; j < n; ++j) u += Q[t * PM + j] * zz[j];
      vv[t] = u;
    }
  } else if (t < 64) {  // EXACT
    // u = H_0 (H_1 (... (H_{n-3} z))), H_k = I - beta_k v_k v_k^T with v_k in
    // column k of A below the diagonal; one wave
    for (int k = n - 3; k >= 0; --k) {
      const double bt = beta[k];
      if (bt == 0.0) continue;  // uniform
      const int m = n - k - 1;
      double sp = 0.0;
      for (int i = lane; i < m; i += 64) sp += A[L(k + 1 + i, k)] * zz[k + 1 + i];
      const double sc = bt * wave_sum(sp);
      for (int i = lane; i < m; i += 64) zz[k + 1 + i] -= sc * A[L(k + 1 + i, k)];
      __builtin_amdgcn_wave_barrier();  // the next step reads other lanes' updates
    }
    for (int i = lane; i < n; i += 64) vv[i] = zz[i];
  }
  __syncthreads();
  // guess 0: the P-space eigenvector u; guess 1: the dense vector
  // r = sign/sqrt(ndet) minus its component on u (u lives on the P block),
  // |r - c u|^2 = 1 - c^2
  double* __restrict__ v0 = V + I.off;
  for (int k = t; k < n; k += NT) v0[idx[k]] = vv[k];
  if (t == 0) {
    const double rs = 1.0 / sqrt((double)nd);
    double c0 = 0.0;
    for (int k = 0; k < n; ++k) c0 += vv[k] * hash_sign(idx[k]) * rs;
    zz[0] = c0;
    zz[2] = 1.0 - c0 * c0;
  }
  __syncthreads();
  const bool dense = nd > n && zz[2] > 1e-6;
  if (dense) {
    const double rs = 1.0 / sqrt((double)nd), rn = 1.0 / sqrt(zz[2]);
    double* __restrict__ vr = V + ntot + I.off;
    for (int64_t K = t; K < nd; K += NT) vr[K] = hash_sign(K) * rs * rn;
    __syncthreads();   // the P-block entries below overwrite the dense pass
    for (int k = t; k < n; k += NT)
      vr[idx[k]] = (hash_sign(idx[k]) * rs - zz[0] * vv[k]) * rn;
  }
  if (t == 0) {
    S.m = 0;
    S.nguess = 1 + (dense ? 1 : 0);
    S.np = EXACT ? 0 : n;  // an exact guess needs no P-space correction
    S.onepass = 0;
    S.olsen = 0;
    S.iters = 0;
    S.status = 0;
    S.rnorm = 0.0;
    S.conv = 0;
    S.theta = 0.0;
  }
}

// P-space correction, run after k_dav_residual: on the P block replace the
// diagonal correction by t_P = Q (theta - T)^-1 Q^T r_P = (theta - H_PP)^-1 r_P,
// and store the change of the Gram-Schmidt dots V_i . t (i < m) and of |t|^2
// in pdots[item][0..kMaxSpace] for k_dav_reduce1.
__global__ void __launch_bounds__(256) k_pspace_correct(const Item* __restrict__ items, int ibase,
                                                        const int32_t* __restrict__ pidx,
                                                        const double* __restrict__ pQ,
                                                        const double* __restrict__ pT, double* V,
                                                        const double* __restrict__ Sv,
                                                        int64_t ntot,
                                                        const DavState* __restrict__ st,
                                                        double* __restrict__ pdots) {
  constexpr int PM = kMaxPspace;
  const int it = ibase + blockIdx.x;
  const Item& I = items[it];
  const DavState& S = st[it];
  if (S.conv || S.np == 0 || S.olsen) return;
  const int np = S.np, m = S.m, t = threadIdx.x;
  const double th = S.theta;
  __shared__ double r[PM], z[PM], dd[PM], ee[PM], piv[PM];
  const int32_t* __restrict__ idx = pidx + (int64_t)it * PM;
  const double* __restrict__ Qi = pQ + (int64_t)it * PM * PM;
  double tnew = 0.0, told = 0.0;
  int e = 0;
  if (t < np) {
    e = idx[t];
    double rv = 0.0;
    for (int i = 0; i < m; ++i)
      rv += S.y[i] * (Sv[(int64_t)i * ntot + I.off + e] - th * V[(int64_t)i * ntot + I.off + e]);
    r[t] = rv;
    told = V[(int64_t)m * ntot + I.off + e];
    dd[t] = pT[(int64_t)it * 2 * PM + t];
    ee[t] = pT[(int64_t)it * 2 * PM + PM + t];
  }
  __syncthreads();
  if (t < np) {
    double zj = 0.0;
    for (int k = 0; k < np; ++k) zj += Qi[k * PM + t] * r[k];
    z[t] = zj;
  }
  __syncthreads();
  if (t == 0) tridiag_shift_solve(dd, ee, np, th, z, z, piv, 1e-8);
  __syncthreads();
  double acc[kMaxSpace + 1];
#pragma unroll
  for (int i = 0; i <= kMaxSpace; ++i) acc[i] = 0.0;
  if (t < np) {
    for (int j = 0; j < np; ++j) tnew += Qi[t * PM + j] * z[j];
    V[(int64_t)m * ntot + I.off + e] = tnew;
    const double dl = tnew - told;
#pragma unroll
    for (int i = 0; i < kMaxSpace; ++i)
      if (i < m) acc[i] = V[(int64_t)i * ntot + I.off + e] * dl;
    acc[kMaxSpace] = tnew * tnew - told * told;
  }
  block_reduce_store<kMaxSpace + 1>(acc, pdots + (int64_t)it * (kMaxSpace + 1));
}

// ------------------------------------------------------------------- RDMs
// For a converged CASCI vector c (normalised):
//   gamma+_ab  = sum_K c_K D+_ab[K]            (= 2 gamma_ab for a > b, gamma_aa)
//   Gamma+_{ab,cd} = sum_K D+_ab[K] D+_cd[K]   (a symmetric rank-update on FP64 MFMA)
// with gamma_pq = <E_pq>, Gamma_pqrs = <E_pq E_rs> - d_qr gamma_ps.  The CI
// vector itself is carried as row NP of the D+ tile (a padding row), so
// gamma+ is column NP of Gamma+ and Gamma+_{NP,NP} = |c|^2.  Each workgroup
// accumulates the upper 16x16 blocks over its tiles in registers and writes
// one partial; k_rdm_reduce sums the partials in a fixed order.
template <int NACT, int TN>
__global__ void __launch_bounds__(256) k_rdm_syrk(const Item* __restrict__ items,
                                                  const Work* __restrict__ work,
                                                  const double* __restrict__ civ,
                                                  double* __restrict__ part) {
  constexpr int NP = NACT * (NACT + 1) / 2;
  constexpr int KPAD = (NP + 15) / 16 * 16;
  constexpr int NRB = KPAD / 16;
  constexpr int NBLK = NRB * (NRB + 1) / 2;   // upper 16x16 blocks
  constexpr int BPW = (NBLK + 3) / 4;         // blocks per wave
  constexpr int NSUB = 256 / TN;
  constexpr int NPER = (NP + NSUB - 1) / NSUB;
  constexpr int LDT = TN + 1;
  constexpr int CMAX = (int)binom_c(NACT, NACT / 2);
  static_assert(NP < KPAD, "the c row needs a padding row");
  __shared__ double Ds[KPAD * LDT];
  __shared__ int32_t Tb[NP * TN];
  __shared__ double Cr[CMAX];

  const Work wk = work[blockIdx.x];
  const Item& I = items[wk.item];
  const double* __restrict__ c = civ + I.off;
  const int Na = I.Na, Nb = I.Nb;
  const int32_t* __restrict__ pA = I.pairA;
  const int32_t* __restrict__ pB = I.pairB;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int col = t % TN;
  const int sub = (TN >= 64) ? __builtin_amdgcn_readfirstlane(t / TN) : t / TN;
  const int blk = wk.begin / Na;
  const int Kb0 = blk * TN;
  const int Kb = Kb0 + col;
  const double keep = Kb < Nb ? 1.0 : 0.0;
  const int Kbc = Kb < Nb ? Kb : Nb - 1;
  for (int x = t; x < NP * TN; x += 256) {
    const int ab = x / TN, cc = x - ab * TN;
    const int kb = Kb0 + cc < Nb ? Kb0 + cc : Nb - 1;
    Tb[x] = ldg(pB + ab * Nb + kb);
  }
  for (int x = (NP + 1) * LDT + t; x < KPAD * LDT; x += 256) Ds[x] = 0.0;
  // this wave's output blocks (rb <= cb) in a fixed enumeration
  int brb[BPW], bcb[BPW];
  double4_t acc[BPW];
#pragma unroll
  for (int u = 0; u < BPW; ++u) {
    int id = wave + 4 * u, rb = 0;
    while (id >= NRB - rb && rb < NRB) { id -= NRB - rb; ++rb; }
    brb[u] = rb;
    bcb[u] = rb + id;
    acc[u] = (double4_t){0.0, 0.0, 0.0, 0.0};
  }
  for (int tile = wk.begin; tile < wk.end; ++tile) {
    const int Ka = tile - blk * Na;
    for (int x = t; x < Nb; x += 256) Cr[x] = ldg(c + Ka * Nb + x);
    __syncthreads();
    const int32_t* __restrict__ pa = pA + Ka * NP;
    const double* __restrict__ ca = c + Kbc;
#pragma unroll
    for (int i = 0; i < NPER; ++i) {
      const int ab = sub + NSUB * i;
      if (ab < NP) {
        const int32_t ea = ldc(pa + ab);
        const int32_t eb = Tb[ab * TN + col];
        const int ja = ea ? (ea >> 1) - 1 : 0, jb = eb ? (eb >> 1) - 1 : 0;
        const double fa = ea ? ((ea & 1) ? -keep : keep) : 0.0;
        const double fb = eb ? ((eb & 1) ? -keep : keep) : 0.0;
        Ds[ab * LDT + col] = fa * ldg(ca + ja * Nb) + fb * Cr[jb];
      }
    }
    if (sub == 0) Ds[NP * LDT + col] = keep * Cr[Kbc];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < BPW; ++u) {
      if (wave + 4 * u >= NBLK) continue;
      const double* ar = Ds + (brb[u] * 16 + (lane & 15)) * LDT + (lane >> 4);
      const double* br = Ds + (bcb[u] * 16 + (lane & 15)) * LDT + (lane >> 4);
#pragma unroll
      for (int k = 0; k < TN; k += 4)
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[k], br[k], acc[u], 0, 0, 0);
    }
    __syncthreads();
  }
  double* out = part + (int64_t)blockIdx.x * KPAD * KPAD;
#pragma unroll
  for (int u = 0; u < BPW; ++u) {
    if (wave + 4 * u >= NBLK) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = brb[u] * 16 + (lane >> 4) + 4 * v, cc = bcb[u] * 16 + (lane & 15);
      out[r * KPAD + cc] = acc[u][v];
    }
  }
}

// Sum the partials of every item in work order; fill the lower triangle.
// rdmp: [item][KPAD*KPAD] (KPAD of that item).
__global__ void k_rdm_reduce(const Item* __restrict__ items, const int32_t* __restrict__ wlo,
                             const int32_t* __restrict__ whi, const double* __restrict__ part,
                             const int64_t* __restrict__ poff, double* rdmp,
                             const int64_t* __restrict__ roff) {
  const int it = blockIdx.x;
  const Item& I = items[it];
  const int kp = I.kpad;
  double* out = rdmp + roff[it];
  for (int x = threadIdx.x; x < kp * kp; x += blockDim.x) {
    const int r = x / kp, cc = x % kp;
    const int rr = r < cc ? r : cc, c2 = r < cc ? cc : r;  // upper triangle holds the data
    double sacc = 0.0;
    if (I.ndet == 1) {
      // single determinant: D+_aa = occupation, c = 1
      sacc = 0.0;
    } else {
      for (int w = wlo[it]; w < whi[it]; ++w) sacc += part[poff[w] + rr * kp + c2];
    }
    out[x] = sacc;
  }
}

// ------------------------------------------------------ gradient assembly
// Weight of f(U) in L = g_0 E_ref + sum_n g_n E^(n): from the closed form
// E^(n) = sum_{|U| <= n} (-1)^{n-|U|} C(M_exp - |U|, n - |U|) f(U), f(()) = E_ref
// (the Moebius solution of the recursion of Eq. 2).
__global__ void k_mbe_weights(const BucketDev* __restrict__ buckets, int nbucket, int nitem,
                              int nexp, int max_order, const double* __restrict__ g, double* w) {
  int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= nitem) return;
  int b = 0;
  while (b + 1 < nbucket && buckets[b + 1].item0 <= it) ++b;
  const int u = buckets[b].order;
  double acc = (u == 0) ? g[0] : 0.0;
  for (int n = (u > 1 ? u : 1); n <= max_order; ++n) {
    const double cb = (double)binom(nexp - u, n - u);
    acc += (((n - u) & 1) ? -cb : cb) * g[n];
  }
  w[it] = acc;
}

// Orbital class of p in CASCI `it`: >= 0 local active index, -1 frozen
// (doubly occupied), -2 deleted.  A single-determinant CASCI has its active
// orbitals either all occupied or all empty and is treated as frozen/deleted.
__device__ inline int orb_class(const int32_t* __restrict__ act, int n, bool single,
                                uint64_t occmask, int p) {
  if (!single)
    for (int t = 0; t < n; ++t)
      if (act[t] == p) return t;
  return (occmask >> p & 1) ? -1 : -2;
}

// gamma_tu of an item from Gamma+ (column NP holds gamma+ = D+ c)
__device__ inline double act_gamma(const double* __restrict__ R, int kp, int np, int t, int u) {
  const double g = R[pair_index(t, u) * kp + np];
  return t == u ? g : 0.5 * g;
}

// 1/4 [G_pqrs + G_qprs + G_pqsr + G_qpsr] of the full-space 2-RDM of one
// CASCI, G = <E_pq E_rs> - d_qr gamma_ps (frozen orbitals doubly occupied).
__device__ double sym_gamma2(int p, int q, int r, int s, int cp, int cq, int cr, int cs,
                             const double* __restrict__ R, int kp, int np) {
  if (cp == -2 || cq == -2 || cr == -2 || cs == -2) return 0.0;
  if (cp >= 0 && cq >= 0 && cr >= 0 && cs >= 0) {
    const double mpq = cp == cq ? 2.0 : 1.0, mrs = cr == cs ? 2.0 : 1.0;
    double v = mpq * mrs * R[pair_index(cp, cq) * kp + pair_index(cr, cs)];
    if (cq == cr) v -= act_gamma(R, kp, np, cp, cs);
    if (cp == cr) v -= act_gamma(R, kp, np, cq, cs);
    if (cq == cs) v -= act_gamma(R, kp, np, cp, cr);
    if (cp == cs) v -= act_gamma(R, kp, np, cq, cr);
    return 0.25 * v;
  }
  // some index frozen: average the raw element over the four index orders
  const int P[4][4] = {{p, q, r, s}, {q, p, r, s}, {p, q, s, r}, {q, p, s, r}};
  const int C[4][4] = {{cp, cq, cr, cs}, {cq, cp, cr, cs}, {cp, cq, cs, cr}, {cq, cp, cs, cr}};
  double acc = 0.0;
  for (int k = 0; k < 4; ++k) {
    const int a = P[k][0], b = P[k][1], c = P[k][2], d = P[k][3];
    const int ca = C[k][0], cb = C[k][1], cc = C[k][2], cd = C[k][3];
    const bool Fa = ca == -1, Fb = cb == -1, Fc = cc == -1, Fd = cd == -1;
    const bool Aa = ca >= 0, Ab = cb >= 0, Ac = cc >= 0, Ad = cd >= 0;
    double v = 0.0;
    if (Fa && Fb && Fc && Fd) {
      if (a == b && c == d) v = (a == c) ? 2.0 : 4.0;
      else if (a == d && b == c) v = -2.0;
    } else if (Fa && Fb && a == b && Ac && Ad) {
      v = 2.0 * act_gamma(R, kp, np, cc, cd);
    } else if (Fc && Fd && c == d && Aa && Ab) {
      v = 2.0 * act_gamma(R, kp, np, ca, cb);
    } else if (Fb && Fc && b == c && Aa && Ad) {
      v = -act_gamma(R, kp, np, ca, cd);
    } else if (Fa && Fd && a == d && Ab && Ac) {
      v = -act_gamma(R, kp, np, cc, cb);
    }
    acc += v;
  }
  return 0.25 * acc;
}

// Sum over a wave by a butterfly: every lane ends with the same value, and
// the order of the additions is fixed by the lane numbering alone.
__device__ inline double wave_sum64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Orbitals on which a CASCI's full-space RDMs can be non-zero: its active
// orbitals and the occupied orbitals of the reference determinant (frozen
// when not active); every other orbital is deleted.  A single-determinant
// CASCI counts only the occupied ones (its active orbitals are frozen or
// deleted alike).  One thread per item.
__global__ void k_grad_masks(const Item* __restrict__ items, int nitem,
                             const int32_t* __restrict__ act, uint64_t occmask,
                             uint64_t* __restrict__ live) {
  const int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= nitem) return;
  const Item& I = items[it];
  uint64_t m = occmask;
  if (I.ndet > 1)
    for (int t = 0; t < I.n; ++t) m |= (uint64_t)1 << act[it * kMaxActive + t];
  live[it] = m;
}

// Inverted index: list[v * nitem + k], k < count[v], the items whose live
// mask holds orbital v, in ascending order (one wave per orbital compacts
// the items with a ballot, so the order is fixed).
__global__ void __launch_bounds__(64) k_grad_index(const uint64_t* __restrict__ live, int nitem,
                                                   int32_t* __restrict__ list,
                                                   int32_t* __restrict__ count) {
  const int v = blockIdx.x, lane = threadIdx.x;
  int base = 0;
  for (int it0 = 0; it0 < nitem; it0 += 64) {
    const int it = it0 + lane;
    const bool has = it < nitem && ((live[it] >> v) & 1);
    const uint64_t b = __ballot(has);
    if (has) list[(int64_t)v * nitem + base + __popcll(b & ((1ull << lane) - 1))] = it;
    base += __popcll(b);
  }
  if (lane == 0) count[v] = base;
}

// Inverted lists of orbital pairs u < v (pair number v (v - 1) / 2 + u):
// the items whose live mask holds both, in ascending order, stored one after
// another (pair p at poff[p], pcount[p] entries).  An element with two or
// more distinct orbitals draws on the shortest of its pairs' lists when that
// is shorter than its orbitals' lists: the items that hold two given
// expansion orbitals are far fewer than those that hold one.
__host__ __device__ inline int orb_pair_id(int u, int v) { return v * (v - 1) / 2 + u; }

// pcount of pair (blockIdx.x, blockIdx.y) when x < y; one wave per pair.
__global__ void __launch_bounds__(64) k_grad_pair_count(const uint64_t* __restrict__ live,
                                                        int nitem, int32_t* __restrict__ pcount) {
  const int u = blockIdx.x, v = blockIdx.y, lane = threadIdx.x;
  if (u >= v) return;
  const uint64_t m = ((uint64_t)1 << u) | ((uint64_t)1 << v);
  int n = 0;
  for (int it0 = 0; it0 < nitem; it0 += 64) {
    const int it = it0 + lane;
    n += __popcll(__ballot(it < nitem && (live[it] & m) == m));
  }
  if (lane == 0) pcount[orb_pair_id(u, v)] = n;
}

// poff[p] = pcount[0] + ... + pcount[p - 1] for p <= npair: one wave, lane
// l sums a contiguous chunk, the chunk sums are scanned across the lanes.
__global__ void __launch_bounds__(64) k_grad_pair_scan(const int32_t* __restrict__ pcount,
                                                       int npair, int64_t* __restrict__ poff) {
  const int lane = threadIdx.x;
  const int per = (npair + 63) / 64;
  const int lo = min(lane * per, npair), hi = min(lo + per, npair);
  int64_t sum = 0;
  for (int i = lo; i < hi; ++i) sum += pcount[i];
  int64_t incl = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  int64_t run = incl - sum;
  for (int i = lo; i < hi; ++i) {
    poff[i] = run;
    run += pcount[i];
  }
  if (lane == 63) poff[npair] = incl;
}

// The list of pair (blockIdx.x, blockIdx.y), x < y, compacted with a ballot
// in ascending item order; one wave per pair.
__global__ void __launch_bounds__(64) k_grad_pair_fill(const uint64_t* __restrict__ live,
                                                       int nitem, const int64_t* __restrict__ poff,
                                                       int32_t* __restrict__ plist) {
  const int u = blockIdx.x, v = blockIdx.y, lane = threadIdx.x;
  if (u >= v) return;
  const uint64_t m = ((uint64_t)1 << u) | ((uint64_t)1 << v);
  int32_t* __restrict__ out = plist + poff[orb_pair_id(u, v)];
  int base = 0;
  for (int it0 = 0; it0 < nitem; it0 += 64) {
    const int it = it0 + lane;
    const bool has = it < nitem && (live[it] & m) == m;
    const uint64_t b = __ballot(has);
    if (has) out[base + __popcll(b & ((1ull << lane) - 1))] = it;
    base += __popcll(b);
  }
}

struct GradLists {
  const uint64_t* live;
  const int32_t* list;    // [M][nitem] per-orbital lists
  const int32_t* count;   // [M]
  const int32_t* plist;   // pair lists, concatenated
  const int64_t* poff;    // [npair + 1]
  const int32_t* pcount;  // [npair]
};

// The candidate items of an element with orbitals in mask e: the shortest of
// the inverted lists of its orbitals (ties: the lower orbital) and of its
// orbital pairs (ties: a single orbital, then the earlier pair in
// (lower, higher) order); an item of that list contributes only if its live
// mask holds all of e.  Wave-uniform.
__device__ inline const int32_t* grad_candidates(uint64_t e, int nitem, const GradLists& L,
                                                 int* ncand) {
  int o[4], d = 0;
  for (uint64_t m = e; m; m &= m - 1) o[d++] = __builtin_ctzll(m);
  int best = o[0], nb = L.count[o[0]];
  for (int i = 1; i < d; ++i)
    if (L.count[o[i]] < nb) best = o[i], nb = L.count[o[i]];
  const int32_t* cand = L.list + (int64_t)best * nitem;
  for (int i = 0; i < d; ++i)
    for (int j = i + 1; j < d; ++j) {
      const int pid = orb_pair_id(o[i], o[j]);
      const int np = L.pcount[pid];
      if (np < nb) nb = np, cand = L.plist + L.poff[pid];
    }
  *ncand = nb;
  return cand;
}

// Row and column of entry x of a lower triangle numbered row by row
// (x = i (i + 1) / 2 + j, j <= i).
__device__ inline void tri_index(int64_t x, int* i, int* j) {
  int a = (int)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
  while ((int64_t)a * (a + 1) / 2 > x) --a;
  while ((int64_t)(a + 1) * (a + 2) / 2 <= x) ++a;
  *i = a;
  *j = (int)(x - (int64_t)a * (a + 1) / 2);
}

// dE/dh_pq = sum_it w_it gamma_full(p, q), for p >= q, written to (p, q)
// and (q, p).  One wave per element: lane l sums the candidate items l,
// l + 64, ... (in ascending item order), then the lanes' sums meet in
// wave_sum64 (a fixed order, so the result is bitwise reproducible).
__global__ void __launch_bounds__(64) k_grad_h(const Item* __restrict__ items, int nitem,
                                               const int32_t* __restrict__ act, uint64_t occmask,
                                               int M, const double* __restrict__ w,
                                               const double* __restrict__ rdmp,
                                               const int64_t* __restrict__ roff, GradLists L,
                                               double* out) {
  int p, q;
  tri_index(blockIdx.x, &p, &q);
  const int lane = threadIdx.x;
  const uint64_t e = ((uint64_t)1 << p) | ((uint64_t)1 << q);
  int nv;
  const int32_t* __restrict__ cand = grad_candidates(e, nitem, L, &nv);
  double acc = 0.0;
  for (int k = lane; k < nv; k += 64) {
    const int it = cand[k];
    if (e & ~L.live[it]) continue;
    const double wt = w[it];
    if (wt == 0.0) continue;
    const Item& I = items[it];
    const bool single = I.ndet == 1;
    const int32_t* a = act + it * kMaxActive;
    const int cp = orb_class(a, I.n, single, occmask, p), cq = orb_class(a, I.n, single, occmask, q);
    double val = 0.0;
    if (cp == -1 && cq == -1 && p == q) val = 2.0;
    else if (cp >= 0 && cq >= 0) val = act_gamma(rdmp + roff[it], I.kpad, I.npair, cp, cq);
    acc += wt * val;
  }
  acc = wave_sum64(acc);
  if (lane == 0) {
    out[p * M + q] = acc;
    out[q * M + p] = acc;
  }
}

// dE/d(pq|rs) = sum_it w_it 1/2 Sym8(Gamma_full)_pqrs.  The value has the
// 8-fold symmetry of the integrals, so it is formed once per orbit (p >= q,
// r >= s, pair pq >= pair rs) and written to all eight positions; one wave
// per orbit as in k_grad_h (four per 256-thread block).  An element with an
// orbital outside every CASCI's live set, or with more expansion orbitals
// than any tuple holds, finds an empty or non-matching candidate list.
__global__ void __launch_bounds__(256) k_grad_g(const Item* __restrict__ items, int nitem,
                                                const int32_t* __restrict__ act, uint64_t occmask,
                                                int M, const double* __restrict__ w,
                                                const double* __restrict__ rdmp,
                                                const int64_t* __restrict__ roff, GradLists L,
                                                double* out) {
  const int64_t x = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t np = (int64_t)M * (M + 1) / 2;
  if (x >= np * (np + 1) / 2) return;  // whole waves
  int P, Q, p, q, r, s;
  tri_index(x, &P, &Q);
  tri_index(P, &p, &q);
  tri_index(Q, &r, &s);
  const uint64_t e = ((uint64_t)1 << p) | ((uint64_t)1 << q) | ((uint64_t)1 << r) |
                     ((uint64_t)1 << s);
  int nv;
  const int32_t* __restrict__ cand = grad_candidates(e, nitem, L, &nv);
  double acc = 0.0;
  for (int k = lane; k < nv; k += 64) {
    const int it = cand[k];
    if (e & ~L.live[it]) continue;
    const double wt = w[it];
    if (wt == 0.0) continue;
    const Item& I = items[it];
    const bool single = I.ndet == 1;
    const int32_t* a = act + it * kMaxActive;
    const int cp = orb_class(a, I.n, single, occmask, p);
    const int cq = orb_class(a, I.n, single, occmask, q);
    const int cr = orb_class(a, I.n, single, occmask, r);
    const int cs = orb_class(a, I.n, single, occmask, s);
    acc += wt * 0.5 * sym_gamma2(p, q, r, s, cp, cq, cr, cs, rdmp + roff[it], I.kpad, I.npair);
  }
  acc = wave_sum64(acc);
  if (lane < 8) {
    // lane l writes the permutation (bit 0: swap p q, bit 1: swap r s, bit 2: swap the pairs)
    int a = p, b = q, c = r, d = s;
    if (lane & 1) a = q, b = p;
    if (lane & 2) c = s, d = r;
    if (lane & 4) {
      const int t0 = a, t1 = b;
      a = c, b = d, c = t0, d = t1;
    }
    out[(((int64_t)a * M + b) * M + c) * M + d] = acc;
  }
}

// RDMs of one whole-space CASCI: rdm1 = gamma, rdm2 = Sym8(Gamma).
__global__ void k_casci_rdm_out(const Item* __restrict__ items, int it,
                                const double* __restrict__ rdmp, const int64_t* __restrict__ roff,
                                double* rdm1, double* rdm2) {
  const Item& I = items[it];
  const int n = I.n;
  const double* R = rdmp + roff[it];
  const int64_t n2 = (int64_t)n * n;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n2 * n2;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(x / (n2 * n)), q = (int)((x / n2) % n), r = (int)((x / n) % n),
              s = (int)(x % n);
    if (rdm2) {
      double v;
      if (I.ndet == 1) {
        // every active orbital doubly occupied (nalpha = nbeta = n) or empty
        const bool full = I.na == n;
        v = 0.0;
        if (full) {
          if (p == q && r == s) v = (p == r) ? 2.0 : 4.0;
          else if (p == s && q == r) v = -1.0;  // Sym8 of -2 over the (ij|ji) orbit
          else if ((p == r && q == s) && p != q) v = -1.0;
        }
      } else {
        v = sym_gamma2(p, q, r, s, p, q, r, s, R, I.kpad, I.npair);
      }
      rdm2[x] = v;
    }
    if (rdm1 && x < n2) {
      const int a = (int)(x / n), b = (int)(x % n);
      rdm1[x] = I.ndet == 1 ? ((a == b && I.na == n) ? 2.0 : 0.0)
                            : act_gamma(R, I.kpad, I.npair, a, b);
    }
  }
}

// ---------------------------------------------------------- MBE combine
// f(T) = E_core(T) + theta_T ; eps_T = f(T) - E_ref ;
// Delta eps_T = sum over non-empty U in T of (-1)^{|T|-|U|} eps_U, which is the
// solution of the recursion of Eq. 2 (Moebius inversion of
// eps_T = sum_{non-empty U in T} Delta eps_U).
__global__ void k_item_energy(const Item* __restrict__ items, const ItemHam* __restrict__ hams,
                              const DavState* __restrict__ st, int nitem, double* f) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nitem) return;
  f[i] = hams[items[i].ham].ecore + st[i].theta;
}

__global__ void k_mbe_increments(MbeSpaces sp, const BucketDev* __restrict__ buckets, int nbucket,
                                 const int32_t* __restrict__ tuple_pos, int max_order,
                                 const double* __restrict__ f, int nitem, double* inc,
                                 double* inc_lex, double* f_lex,
                                 const int64_t* __restrict__ order_off,
                                 const int32_t* __restrict__ xpos_o,
                                 const int32_t* __restrict__ xpos_v, int nX) {
  int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= nitem || it == 0) return;   // item 0 is the reference CASCI
  const int32_t* tp = tuple_pos + (int64_t)it * (2 * max_order + 2);
  const int no = tp[0], nv = tp[1], n = no + nv;
  const double eref = f[0];
  // bucket base index per (order, nocc)
  double acc = 0.0;
  const unsigned full = (1u << n) - 1u;
  for (unsigned sub = 1; sub <= full; ++sub) {
    int co[kMaxActive], cv[kMaxActive];
    int ko = 0, kv = 0;
    for (int b = 0; b < n; ++b)
      if (sub >> b & 1) {
        if (b < no) co[ko++] = tp[2 + b];
        else cv[kv++] = tp[2 + b];
      }
    const int ord = ko + kv;
    int64_t base = -1;
    for (int b = 0; b < nbucket; ++b)
      if (buckets[b].order == ord && buckets[b].nocc == ko) base = buckets[b].item0;
    const int64_t idx = base + comb_lex_rank(co, ko, sp.nXo) * binom(sp.nXv, kv) +
                        comb_lex_rank(cv, kv, sp.nXv);
    const double e = f[idx] - eref;
    acc += ((n - ord) & 1) ? -e : e;
  }
  inc[it] = acc;
  if (inc_lex) {
    // lexicographic rank of T among the order-n tuples of the sorted X
    int c[kMaxActive];
    for (int b = 0; b < no; ++b) c[b] = xpos_o[tp[2 + b]];
    for (int b = 0; b < nv; ++b) c[no + b] = xpos_v[tp[2 + no + b]];
    for (int a = 1; a < n; ++a) {
      int v = c[a], j = a - 1;
      while (j >= 0 && c[j] > v) { c[j + 1] = c[j]; --j; }
      c[j + 1] = v;
    }
    const int64_t lx = order_off[n - 1] + comb_lex_rank(c, n, nX);
    inc_lex[lx] = acc;
    if (f_lex) f_lex[lx] = f[it];
  }
}

// E^(n) = sum of the order-n increments, one block per order, fixed order.
__global__ void k_mbe_order_sums(const BucketDev* __restrict__ buckets, int nbucket,
                                 const double* __restrict__ inc, double* e_order) {
  const int n = blockIdx.x + 1;
  __shared__ double red[256];
  double acc = 0.0;
  for (int b = 0; b < nbucket; ++b) {
    if (buckets[b].order != n) continue;
    for (int64_t i = threadIdx.x; i < buckets[b].count; i += 256) acc += inc[buckets[b].item0 + i];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) e_order[n - 1] = red[0];
}

// ------------------------------------------------------- bookkeeping kernels
// number of items of [ibase, ibase+nitem) not yet converged (one block)
__global__ void k_count_active(const DavState* __restrict__ st, int ibase, int nitem, int* out) {
  __shared__ int red[256];
  int c = 0;
  for (int i = threadIdx.x; i < nitem; i += 256) c += st[ibase + i].conv ? 0 : 1;
  red[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// per-item (iterations, status, guess count, subspace) for the statistics
__global__ void k_collect(const DavState* __restrict__ st, int nitem, int32_t* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nitem) return;
  out[4 * i + 0] = st[i].iters;
  out[4 * i + 1] = st[i].status;
  out[4 * i + 2] = st[i].nguess;
  out[4 * i + 3] = st[i].conv;
}

// state of a single caller-provided vector in slot 0 (sigma entry point)
__global__ void k_state_single(DavState* st) {
  if (threadIdx.x == 0) {
    st->m = 1;
    st->nguess = 1;
    st->conv = 0;
    st->iters = 0;
    st->status = 0;
  }
}

// mark every multi-determinant item unconverged (kernel re-timing)
__global__ void k_state_unconv(const Item* __restrict__ items, DavState* st, int nitem) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nitem && items[i].ndet > 1) st[i].conv = 0;
}

// out = s + a*c
__global__ void k_axpy_out(double* out, const double* s, const double* c, double a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = s[i] + a * c[i];
}

// out = (d + a) * c  (sigma of a diagonal Hamiltonian)
__global__ void k_diag_times(double* out, const double* d, const double* c, double a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (d[i] + a) * c[i];
}

__global__ void k_add_scalar(double* out, const double* in, double a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i] + a;
}

// Ritz vector x = V y of every item into `out` (arena layout), normalised.
__global__ void __launch_bounds__(256) k_ritz_vector(const Item* __restrict__ items,
                                                     const Work* __restrict__ work,
                                                     const double* __restrict__ V, int64_t ntot,
                                                     const DavState* __restrict__ st,
                                                     double* out) {
  const Work wk = work[blockIdx.x];
  const Item& I = items[wk.item];
  const DavState& S = st[wk.item];
  const int64_t e0 = (int64_t)(wk.begin - I.chunk0) * kChunk;
  const int64_t e1 = min(e0 + kChunk, I.ndet);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    double x = 0.0;
    if (I.ndet == 1) {
      x = 1.0;
    } else {
      for (int i = 0; i < S.m; ++i) x += S.y[i] * V[(int64_t)i * ntot + I.off + e];
    }
    out[I.off + e] = x;
  }
}

// E_total = E_ref + sum_n E^(n), in order
__global__ void k_mbe_total(const double* f, const double* e_order, int k, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double e = f[0];
    for (int n = 0; n < k; ++n) e += e_order[n];
    out[0] = f[0];
    out[1] = e;
  }
}

// ------------------------------------------------------- screened expansion
// Set-up from explicit tuples: item i holds the tuple with orbital mask
// masks[i] (bit p = expansion orbital p of the problem; 0 = the reference
// CASCI of R alone).  A = R u T, F = O \ A frozen, the rest deleted.
__global__ void k_mbe_setup_list(MbeSpaces sp, const uint64_t* __restrict__ masks,
                                 const Item* __restrict__ items, const double* __restrict__ h1,
                                 const double* __restrict__ eri, double e_const, ItemHam* hams,
                                 double* warena) {
  const int it = blockIdx.x;
  __shared__ ActiveSet s;
  if (threadIdx.x == 0) {
    const uint64_t m = masks[it];
    uint64_t a = m;
    for (int i = 0; i < sp.nR; ++i) a |= (uint64_t)1 << sp.R[i];
    int nt = 0;
    for (uint64_t x = a; x; x &= x - 1) s.act[nt++] = __builtin_ctzll(x);  // ascending
    s.n = nt;
    s.nf = 0;
    int na = 0;
    for (int i = 0; i < sp.nO; ++i) {
      const int o = sp.O[i];
      if (a >> o & 1) ++na;
      else s.frz[s.nf++] = o;
    }
    s.na = na;
  }
  __syncthreads();
  const Item& I = items[it];
  build_item_hamiltonian(s, sp.M, h1, eri, e_const, I.na + I.nb, &hams[I.ham],
                         I.ndet > 1 ? warena + I.woff : nullptr, I.kpad);
}

// Computed tuples of the lower orders, each order's masks in ascending
// numeric order with their increments.
struct ScreenLevels {
  const uint64_t* mask[kMaxActive + 1];
  const double* inc[kMaxActive + 1];
  int64_t n[kMaxActive + 1];
};

// Eq. 2 over the computed sub-tuples: for tuple i of order k,
// Delta eps = (f_i - E_ref) - sum over its proper non-empty sub-tuples U that
// were computed of Delta eps_U (binary search in U's order; sub-tuples in
// ascending subset order, so the sum has a fixed order).
__global__ void k_screen_increments(const uint64_t* __restrict__ masks, int64_t n, int k,
                                    const double* __restrict__ f, const double* __restrict__ e_ref,
                                    ScreenLevels lv, double* __restrict__ inc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t m = masks[i];
  int bit[kMaxActive];
  int nb = 0;
  for (uint64_t x = m; x; x &= x - 1) bit[nb++] = __builtin_ctzll(x);
  double d = f[i] - e_ref[0];
  const uint32_t full = (1u << k) - 1u;
  for (uint32_t sub = 1; sub < full; ++sub) {
    uint64_t u = 0;
    for (int b = 0; b < k; ++b)
      if (sub >> b & 1) u |= (uint64_t)1 << bit[b];
    const int o = __builtin_popcount(sub);
    const uint64_t* __restrict__ arr = lv.mask[o];
    int64_t lo = 0, hi = lv.n[o];
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (arr[mid] < u) lo = mid + 1;
      else hi = mid;
    }
    if (lo < lv.n[o] && arr[lo] == u) d -= lv.inc[o][lo];
  }
  inc[i] = d;
}

// E^(k) = sum of the order-k increments, in index order (one thread).
// E^(k): one block, every thread a strided partial sum, then a fixed-order
// wave and block reduction (the order depends only on n, so the result is
// reproducible).
__global__ void __launch_bounds__(1024) k_screen_order_sum(const double* __restrict__ inc,
                                                           int64_t n, double* out) {
  __shared__ double part[16];
  const int t = threadIdx.x;
  double e = 0.0;
  for (int64_t i = t; i < n; i += 1024) e += inc[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) e += __shfl_down(e, o, 64);
  if ((t & 63) == 0) part[t >> 6] = e;
  __syncthreads();
  if (t == 0) {
    double sum = 0.0;
    for (int w = 0; w < 16; ++w) sum += part[w];
    out[0] = sum;
  }
}

// ================================================================ launchers
static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

void launch_strings(int n, int ne, int64_t N, uint64_t* out, hipStream_t s) {
  if (N > 0) hipLaunchKernelGGL(k_strings, dim3(nblk(N, 256)), dim3(256), 0, s, n, ne, N, out);
}
void launch_links(int n, int ne, int64_t N, uint32_t* packed, uint32_t* packedT, int32_t* abi4,
                  hipStream_t s) {
  if (N > 0)
    hipLaunchKernelGGL(k_links, dim3(nblk(N, 128)), dim3(128), 0, s, n, ne, N, packed, packedT,
                       abi4);
}
void launch_pair_table(int n, int ne, int64_t N, int32_t* out, int32_t* outT, hipStream_t s) {
  if (N > 0)
    hipLaunchKernelGGL(k_pair_table, dim3(nblk(N, 128)), dim3(128), 0, s, n, ne, N, out, outT);
}
void launch_mbe_setup(const MbeSpaces* sp, const BucketDev* buckets, int nbucket, const Item* items,
                      int nitem, const double* h1, const double* eri, double e_const,
                      ItemHam* hams, double* warena, int32_t* tuple_pos, int max_order,
                      int32_t* act_out, hipStream_t s) {
  hipLaunchKernelGGL(k_mbe_setup, dim3(nitem), dim3(256), 0, s, *sp, buckets, nbucket, items, h1,
                     eri, e_const, hams, warena, tuple_pos, max_order, act_out);
}
void launch_casci_setup(int n, const double* const* h1s, const double* const* eris,
                        const double* ecores, const Item* items, int nitem, ItemHam* hams,
                        double* warena, hipStream_t s) {
  hipLaunchKernelGGL(k_casci_setup, dim3(nitem), dim3(256), 0, s, n, h1s, eris, ecores, items,
                     hams, warena);
}
void launch_hdiag(const Item* items, const Work* work, int nwork, const ItemHam* hams,
                  double* diag, hipStream_t s) {
  if (nwork > 0)
    hipLaunchKernelGGL(k_hdiag, dim3(nwork), dim3(256), 0, s, items, work, hams, diag);
}

template <int NACT, int TN>
static void sigma_dgemm_t(const Item* items, const Work* work, int nwork, const double* warena,
                          const double* V, int64_t ntot, double* G, double* Sv,
                          const DavState* st, int slot, hipStream_t s) {
  if constexpr (NACT > kFoldMax)
    hipLaunchKernelGGL((k_sigma_dgemm_pairrows<NACT, TN>), dim3(nwork), dim3(dgemm_threads(NACT)),
                       0, s, items, work, warena, V, ntot, G, st, slot);
  else
    hipLaunchKernelGGL((k_sigma_dgemm<NACT, TN>), dim3(nwork), dim3(dgemm_threads(NACT)), 0, s,
                       items, work, warena, V, ntot, G, Sv, st, slot);
}

template <int TN>
static bool sigma_dgemm_n(int n, const Item* items, const Work* work, int nwork,
                          const double* warena, const double* V, int64_t ntot, double* G,
                          double* Sv, const DavState* st, int slot, hipStream_t s) {
  switch (n) {
#define MBEFCI_CASE(N) \
  case N: sigma_dgemm_t<N, TN>(items, work, nwork, warena, V, ntot, G, Sv, st, slot, s); return true;
    MBEFCI_CASE(2) MBEFCI_CASE(3) MBEFCI_CASE(4) MBEFCI_CASE(5) MBEFCI_CASE(6) MBEFCI_CASE(7)
    MBEFCI_CASE(10) MBEFCI_CASE(11) MBEFCI_CASE(12)
#undef MBEFCI_CASE
    case 8:  // three-wave workgroups: up to 64 columns
      if constexpr (TN <= 64) { sigma_dgemm_t<8, TN>(items, work, nwork, warena, V, ntot, G, Sv, st, slot, s); return true; }
      return false;
    case 9:
      if constexpr (TN <= 64) { sigma_dgemm_t<9, TN>(items, work, nwork, warena, V, ntot, G, Sv, st, slot, s); return true; }
      return false;
    case 13:
      if constexpr (TN <= 64) { sigma_dgemm_t<13, TN>(items, work, nwork, warena, V, ntot, G, Sv, st, slot, s); return true; }
      return false;
    case 14:
      if constexpr (TN <= 64) { sigma_dgemm_t<14, TN>(items, work, nwork, warena, V, ntot, G, Sv, st, slot, s); return true; }
      return false;
    default: return false;
  }
}

template <int TN>
static bool sigma_dgemm_flat_n(int n, const Item* items, const Work* work, int nwork,
                               const double* warena, const double* V, int64_t ntot, double* G,
                               double* Sv, const DavState* st, int slot, hipStream_t s) {
  switch (n) {
#define MBEFCI_CASE(N)                                                                       \
  case N:                                                                                    \
    hipLaunchKernelGGL((k_sigma_dgemm_flat<N, TN>), dim3(nwork), dim3(256), 0, s, items,     \
                       work, warena, V, ntot, G, Sv, st, slot);                              \
    return true;
    MBEFCI_CASE(2) MBEFCI_CASE(3) MBEFCI_CASE(4) MBEFCI_CASE(5) MBEFCI_CASE(6) MBEFCI_CASE(7)
    MBEFCI_CASE(8) MBEFCI_CASE(9)
#undef MBEFCI_CASE
    default: return false;
  }
}

bool launch_sigma_dgemm(int n, int tn, const Item* items, const Work* work, int nwork,
                        const double* warena, const double* V, int64_t ntot, double* G,
                        double* Sv, const DavState* st, int slot, hipStream_t s) {
  if (nwork <= 0) return true;
  switch (tn) {
    case -32: return sigma_dgemm_flat_n<32>(n, items, work, nwork, warena, V, ntot, G, Sv, st, slot, s);
    case -64: return sigma_dgemm_flat_n<64>(n, items, work, nwork, warena, V, ntot, G, Sv, st, slot, s);
    case 32: return sigma_dgemm_n<32>(n, items, work, nwork, warena, V, ntot, G, Sv, st, slot, s);
    case 64: return sigma_dgemm_n<64>(n, items, work, nwork, warena, V, ntot, G, Sv, st, slot, s);
    case 128:
      // not compiled for n >= 13 (more LDS than one CU holds) nor for the
      // three-wave workgroups of n = 8, 9: the work units must not be built
      // for it (the caller maps such a schedule to 64 columns)
      return sigma_dgemm_n<128>(n, items, work, nwork, warena, V, ntot, G, Sv, st, slot, s);
    default: return false;
  }
}

int sym_npc(int npair_class) { return npair_class <= 0 ? 0 : (npair_class + 15) / 16 * 16; }

bool launch_sigma_sym_dgemm(int npc, const Item* items, const Work* work, int nwork,
                            const double* warena, const double* V, int64_t ntot, double* G,
                            const DavState* st, int slot, hipStream_t s) {
  if (nwork <= 0) return true;
  switch (npc) {
#define MBEFCI_CASE(P, T)                                                                     \
  case P:                                                                                     \
    hipLaunchKernelGGL((k_sigma_sym_dgemm<P, T>), dim3(nwork), dim3(256), 0, s, items, work,  \
                       warena, V, ntot, G, st, slot);                                         \
    return true;
    MBEFCI_CASE(16, 64) MBEFCI_CASE(32, 64) MBEFCI_CASE(48, 64) MBEFCI_CASE(64, 32)
    MBEFCI_CASE(80, 32) MBEFCI_CASE(96, 32) MBEFCI_CASE(112, 32)
#undef MBEFCI_CASE
    default: return false;
  }
}

void launch_sigma_sym_gather(const Item* items, const Work* work, int nwork, const double* G,
                             double* Sv, int64_t ntot, const DavState* st, int slot,
                             hipStream_t s) {
  if (nwork > 0)
    hipLaunchKernelGGL(k_sigma_sym_gather, dim3(nwork), dim3(256), 0, s, items, work, G, Sv, ntot,
                       st, slot);
}

void launch_sigma_gather(const Item* items, const Work* work, int nwork, const double* G,
                         double* Sv, int64_t ntot, const DavState* st, int slot, int lds,
                         hipStream_t s) {
  if (nwork > 0)
    hipLaunchKernelGGL(k_sigma_gather, dim3(nwork), dim3(256), lds, s, items, work, G, Sv, ntot,
                       st, slot);
}

// ------------------------------------------------------- peak probes
// Measurement only, off the solver's path.  k_probe_mfma runs independent
// chains of FP64 16x16x4 MFMAs per wave from registers (no memory traffic);
// the sum is stored only if it equals a value the inputs never produce,
// which keeps the chains live.  k_probe_copy copies 16-byte vectors.
__global__ void __launch_bounds__(256) k_probe_mfma(double* out, int iters, double seed) {
  constexpr int CH = 8;
  double4_t acc[CH];
#pragma unroll
  for (int ch = 0; ch < CH; ++ch) acc[ch] = (double4_t){0.0, 0.0, 0.0, 0.0};
  const double a = seed + threadIdx.x * 1e-3, b = 0.5 * seed + threadIdx.x * 1e-4;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) acc[ch] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[ch], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int ch = 0; ch < CH; ++ch) s += acc[ch][0] + acc[ch][1] + acc[ch][2] + acc[ch][3];
  if (s == -12345.678) out[threadIdx.x] = s;
}
__global__ void __launch_bounds__(256) k_probe_copy(const double2* __restrict__ src,
                                                    double2* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    dst[i] = src[i];
}
constexpr int kProbeMfmaChains = 8;  // the chains of k_probe_mfma
void launch_probe_mfma(double* out, int blocks, int iters, hipStream_t s) {
  hipLaunchKernelGGL(k_probe_mfma, dim3(blocks), dim3(256), 0, s, out, iters, 1.0);
}
double probe_mfma_flops(int blocks, int iters) {
  return (double)blocks * 4.0 * iters * kProbeMfmaChains * 2.0 * 16 * 16 * 4;
}
void launch_probe_copy(const double* src, double* dst, int64_t n, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, s,
                     reinterpret_cast<const double2*>(src), reinterpret_cast<double2*>(dst), n / 2);
}

void launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  int64_t b = nblk(n, 256);
  if (b > 65536) b = 65536;
  hipLaunchKernelGGL(k_fill, dim3((int)b), dim3(256), 0, s, p, n, v);
}
void launch_dav_guess(const Item* items, int ibase, int nitem, const double* diag, double* V,
                      int64_t ntot, DavState* st, int nguess, hipStream_t s) {
  hipLaunchKernelGGL(k_dav_guess, dim3(nitem), dim3(256), 0, s, items, ibase, diag, V, ntot, st,
                     nguess);
}
void launch_dav_dots(const Item* items, const Work* chunks, int nchunk, const double* V,
                     const double* Sv, int64_t ntot, const DavState* st, int slot, double* part,
                     hipStream_t s) {
  if (nchunk > 0)
    hipLaunchKernelGGL(k_dav_dots, dim3(nchunk), dim3(256), 0, s, items, chunks, V, Sv, ntot, st,
                       slot, part);
}
void launch_dav_rr(const Item* items, int ibase, int nitem, const double* part, DavState* st,
                   int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_dav_rr, dim3(nitem), dim3(64), 0, s, items, ibase, part, st, slot);
}
void launch_pspace_setup(const Item* items, int ibase, int nitem, const PspaceLists& pl,
                         const ItemHam* hams, const double* diag, int32_t* pidx, double* pQ,
                         double* pT, double* V, int64_t ntot, DavState* st, int pmax, int nunit,
                         const PspaceSelect& sel, hipStream_t s) {
  if (sel.nwork > 0)
    hipLaunchKernelGGL(k_pspace_select_chunk, dim3(sel.nwork), dim3(256), 0, s, items, sel.work,
                       ibase, nitem, diag, sel.hi, sel.lo, pmax);
  hipLaunchKernelGGL(k_pspace_select, dim3(nitem), dim3(256), 0, s, items, ibase, diag, pidx, pmax,
                     sel.slot, sel.hi, sel.lo);
  hipLaunchKernelGGL(k_pspace_guess, dim3(nitem), dim3(256), 0, s, items, ibase, diag, pidx, V,
                     ntot, st, pmax, nunit);
  if (pl.n[0] > 0)
    hipLaunchKernelGGL((k_pspace_eigen<kMaxPspace, 512, false>), dim3(pl.n[0]), dim3(512), 0, s,
                       items, pl.list[0], hams, diag, pidx, pQ, pT, V, ntot, st, pmax);
  if (pl.n[1] > 0)
    hipLaunchKernelGGL((k_pspace_eigen<kExactSmall, 64, true>), dim3(pl.n[1]), dim3(64), 0, s,
                       items, pl.list[1], hams, diag, pidx, pQ, pT, V, ntot, st, pmax);
  if (pl.n[2] > 0)
    hipLaunchKernelGGL((k_pspace_eigen<kExactMid, 256, true>), dim3(pl.n[2]), dim3(256), 0, s,
                       items, pl.list[2], hams, diag, pidx, pQ, pT, V, ntot, st, pmax);
  if (pl.n[3] > 0)
    hipLaunchKernelGGL((k_pspace_eigen<kMaxPspace, 256, true>), dim3(pl.n[3]), dim3(256), 0, s,
                       items, pl.list[3], hams, diag, pidx, pQ, pT, V, ntot, st, pmax);
  if (pl.n[4] > 0)
    hipLaunchKernelGGL((k_pspace_eigen<kPspaceMid, 512, false>), dim3(pl.n[4]), dim3(512), 0, s,
                       items, pl.list[4], hams, diag, pidx, pQ, pT, V, ntot, st, pmax);
}
void launch_dav_iteration(const Item* items, int ibase, int nitem, const Work* chunks, int nchunk,
                          double* V, double* Sv, const double* diag, int64_t ntot, DavState* st,
                          double* part, double tol, int max_iter, int mmax, double* Rb,
                          double* Xb, const PspaceArgs* ps, bool olsen_all, double olsen_below,
                          hipStream_t s) {
  if (nchunk <= 0) return;
  const int nb = nblk(nitem, 64);
  hipLaunchKernelGGL(k_dav_collapse, dim3(nchunk), dim3(256), 0, s, items, chunks, V, Sv, ntot, st,
                     mmax);
  hipLaunchKernelGGL(k_dav_collapse_state, dim3(nb), dim3(64), 0, s, items, st, ibase, nitem,
                     mmax);
  // Olsen-corrected items first (all of them with olsen_all, else those that
  // switched in an earlier iteration), then the diagonal / P-space path for
  // the others, whose test may switch an item for the next iteration
  if (olsen_all || olsen_below > 0.0) {
    const int all = olsen_all ? 1 : 0;
    hipLaunchKernelGGL(k_dav_residual_olsen, dim3(nchunk), dim3(256), 0, s, items, chunks, V, Sv,
                       diag, ntot, st, Rb, Xb, part, all);
    hipLaunchKernelGGL(k_dav_reduce1_olsen, dim3(nb), dim3(64), 0, s, items, part, st, ibase,
                       nitem, tol, max_iter, all);
    hipLaunchKernelGGL(k_dav_precond_olsen, dim3(nchunk), dim3(256), 0, s, items, chunks, V, diag,
                       ntot, st, Rb, Xb, part, all);
    hipLaunchKernelGGL(k_dav_reduce_coef, dim3(nb), dim3(64), 0, s, items, part, st, ibase, nitem,
                       all);
  }
  if (!olsen_all) {
    hipLaunchKernelGGL(k_dav_residual, dim3(nchunk), dim3(256), 0, s, items, chunks, V, Sv, diag,
                       ntot, st, part);
    if (ps)
      hipLaunchKernelGGL(k_pspace_correct, dim3(nitem), dim3(256), 0, s, items, ibase, ps->pidx,
                         ps->pQ, ps->pT, V, Sv, ntot, st, ps->pdots);
    hipLaunchKernelGGL(k_dav_reduce1, dim3(nb), dim3(64), 0, s, items, part,
                       ps ? ps->pdots : nullptr, st, ibase, nitem, tol, max_iter, olsen_below);
  }
  hipLaunchKernelGGL(k_dav_orth, dim3(nchunk), dim3(256), 0, s, items, chunks, V, ntot, st, part);
  hipLaunchKernelGGL(k_dav_reduce2, dim3(nb), dim3(64), 0, s, items, part, st, ibase, nitem);
  hipLaunchKernelGGL(k_dav_orth2, dim3(nchunk), dim3(256), 0, s, items, chunks, V, ntot, st);
  hipLaunchKernelGGL(k_dav_grow, dim3(nb), dim3(64), 0, s, st, ibase, nitem);
}
void launch_item_energy(const Item* items, const ItemHam* hams, const DavState* st, int nitem,
                        double* f, hipStream_t s) {
  hipLaunchKernelGGL(k_item_energy, dim3(nblk(nitem, 64)), dim3(64), 0, s, items, hams, st, nitem,
                     f);
}
void launch_mbe_combine(const MbeSpaces* sp, const BucketDev* buckets, int nbucket,
                        const int32_t* tuple_pos, int max_order, const double* f, int nitem,
                        double* inc, double* inc_lex, double* f_lex, const int64_t* order_off,
                        const int32_t* xpos_o, const int32_t* xpos_v, int nX, double* e_order,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_mbe_increments, dim3(nblk(nitem, 64)), dim3(64), 0, s, *sp, buckets,
                     nbucket, tuple_pos, max_order, f, nitem, inc, inc_lex, f_lex, order_off,
                     xpos_o, xpos_v, nX);
  if (max_order > 0)
    hipLaunchKernelGGL(k_mbe_order_sums, dim3(max_order), dim3(256), 0, s, buckets, nbucket, inc,
                       e_order);
}

}  // namespace mbefci

namespace mbefci {
void launch_count_active(const DavState* st, int ibase, int nitem, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_count_active, dim3(1), dim3(256), 0, s, st, ibase, nitem, out);
}
void launch_collect(const DavState* st, int nitem, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_collect, dim3(nblk(nitem, 64)), dim3(64), 0, s, st, nitem, out);
}
void launch_state_single(DavState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_state_single, dim3(1), dim3(64), 0, s, st);
}
void launch_axpy_out(double* out, const double* sv, const double* c, double a, int64_t n,
                     hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_axpy_out, dim3(nblk(n, 256)), dim3(256), 0, s, out, sv, c, a, n);
}
void launch_diag_times(double* out, const double* d, const double* c, double a, int64_t n,
                       hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_diag_times, dim3(nblk(n, 256)), dim3(256), 0, s, out, d, c, a, n);
}
void launch_add_scalar(double* out, const double* in, double a, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_add_scalar, dim3(nblk(n, 256)), dim3(256), 0, s, out, in, a, n);
}
void launch_ritz_vector(const Item* items, const Work* chunks, int nchunk, const double* V,
                        int64_t ntot, const DavState* st, double* out, hipStream_t s) {
  if (nchunk > 0)
    hipLaunchKernelGGL(k_ritz_vector, dim3(nchunk), dim3(256), 0, s, items, chunks, V, ntot, st,
                       out);
}
void launch_state_unconv(const Item* items, DavState* st, int nitem, hipStream_t s) {
  hipLaunchKernelGGL(k_state_unconv, dim3(nblk(nitem, 64)), dim3(64), 0, s, items, st, nitem);
}
void launch_mbe_total(const double* f, const double* e_order, int k, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_mbe_total, dim3(1), dim3(64), 0, s, f, e_order, k, out);
}
}  // namespace mbefci

namespace mbefci {
template <int NACT, int TN>
static void rdm_syrk_t(const Item* items, const Work* work, int nwork, const double* civ,
                       double* part, hipStream_t s) {
  hipLaunchKernelGGL((k_rdm_syrk<NACT, TN>), dim3(nwork), dim3(256), 0, s, items, work, civ, part);
}
bool launch_rdm_syrk(int n, int tn, const Item* items, const Work* work, int nwork,
                     const double* civ, double* part, hipStream_t s) {
  if (nwork <= 0) return true;
  if (tn != 64) return false;
  switch (n) {
#define MBEFCI_CASE(N) \
  case N: rdm_syrk_t<N, 64>(items, work, nwork, civ, part, s); return true;
    MBEFCI_CASE(2) MBEFCI_CASE(3) MBEFCI_CASE(4) MBEFCI_CASE(5) MBEFCI_CASE(6) MBEFCI_CASE(7)
    MBEFCI_CASE(8) MBEFCI_CASE(9) MBEFCI_CASE(10) MBEFCI_CASE(11) MBEFCI_CASE(12)
    MBEFCI_CASE(13) MBEFCI_CASE(14)
#undef MBEFCI_CASE
    default: return false;
  }
}
void launch_rdm_reduce(const Item* items, int nitem, const int32_t* wlo, const int32_t* whi,
                       const double* part, const int64_t* poff, double* rdmp, const int64_t* roff,
                       hipStream_t s) {
  if (nitem > 0)
    hipLaunchKernelGGL(k_rdm_reduce, dim3(nitem), dim3(256), 0, s, items, wlo, whi, part, poff,
                       rdmp, roff);
}
void launch_mbe_weights(const BucketDev* buckets, int nbucket, int nitem, int nexp, int max_order,
                        const double* g, double* w, hipStream_t s) {
  hipLaunchKernelGGL(k_mbe_weights, dim3(nblk(nitem, 64)), dim3(64), 0, s, buckets, nbucket, nitem,
                     nexp, max_order, g, w);
}
void launch_grad_index(const Item* items, int nitem, const int32_t* act, uint64_t occmask, int M,
                       uint64_t* live, int32_t* list, int32_t* count, int32_t* pcount,
                       int64_t* poff, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_masks, dim3(nblk(nitem, 64)), dim3(64), 0, s, items, nitem, act,
                     occmask, live);
  hipLaunchKernelGGL(k_grad_index, dim3(M), dim3(64), 0, s, live, nitem, list, count);
  hipLaunchKernelGGL(k_grad_pair_count, dim3(M, M), dim3(64), 0, s, live, nitem, pcount);
  hipLaunchKernelGGL(k_grad_pair_scan, dim3(1), dim3(64), 0, s, pcount, M * (M - 1) / 2, poff);
}
void launch_grad(const Item* items, int nitem, const int32_t* act, uint64_t occmask, int M,
                 const double* w, const double* rdmp, const int64_t* roff, const uint64_t* live,
                 const int32_t* list, const int32_t* count, const int32_t* pcount,
                 const int64_t* poff, int32_t* plist, double* dh, double* dg, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_pair_fill, dim3(M, M), dim3(64), 0, s, live, nitem, poff, plist);
  const GradLists L{live, list, count, plist, poff, pcount};
  const int64_t np = (int64_t)M * (M + 1) / 2;  // p >= q
  hipLaunchKernelGGL(k_grad_h, dim3((int)np), dim3(64), 0, s, items, nitem, act, occmask, M, w,
                     rdmp, roff, L, dh);
  hipLaunchKernelGGL(k_grad_g, dim3(nblk(np * (np + 1) / 2, 4)), dim3(256), 0, s, items, nitem,
                     act, occmask, M, w, rdmp, roff, L, dg);
}
void launch_casci_rdm_out(const Item* items, int it, int n, const double* rdmp,
                          const int64_t* roff, double* rdm1, double* rdm2, hipStream_t s) {
  const int64_t n4 = (int64_t)n * n * n * n;
  int b = nblk(n4, 256);
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_casci_rdm_out, dim3(b), dim3(256), 0, s, items, it, rdmp, roff, rdm1, rdm2);
}
void launch_mbe_setup_list(const MbeSpaces* sp, const uint64_t* masks, const Item* items, int nitem,
                           const double* h1, const double* eri, double e_const, ItemHam* hams,
                           double* warena, hipStream_t s) {
  hipLaunchKernelGGL(k_mbe_setup_list, dim3(nitem), dim3(256), 0, s, *sp, masks, items, h1, eri,
                     e_const, hams, warena);
}
void launch_screen_increments(const uint64_t* masks, int64_t n, int k, const double* f,
                              const double* e_ref, const ScreenArrays& lower, double* inc,
                              double* order_sum, hipStream_t s) {
  ScreenLevels lv{};
  for (int o = 0; o <= kMaxActive; ++o) {
    lv.mask[o] = lower.mask[o];
    lv.inc[o] = lower.inc[o];
    lv.n[o] = lower.n[o];
  }
  if (n > 0)
    hipLaunchKernelGGL(k_screen_increments, dim3(nblk(n, 128)), dim3(128), 0, s, masks, n, k, f,
                       e_ref, lv, inc);
  hipLaunchKernelGGL(k_screen_order_sum, dim3(1), dim3(1024), 0, s, inc, n, order_sum);
}
}  // namespace mbefci
