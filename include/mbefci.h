/*
 * mbefci.h -- C ABI of the MI355X (gfx950) generalized MBE-FCI hot path.
 *
 * The method (Eriksen & Gauss, "Generalized Many-Body Expanded Full
 * Configuration Interaction Theory", arXiv:1910.03527): the MOs are split into
 * a reference space R and an expansion space X (orbitals of either occupancy).
 * For every tuple T of 1..k expansion orbitals one CASCI is solved in the
 * active space R u T; with eps_T = E_CASCI(R u T) - E_ref the increments obey
 * the recursion of Eq. 2, the order sums E^(n) add the increments of order n,
 * and E_FCI ~ E_ref + sum_n E^(n) (Eq. 1; Eq. 3 for an empty R).
 *
 * Conventions for every call:
 *  - Energies in hartree, FP64.  Orbital indices 0-based.  Arrays row-major.
 *    Two-electron integrals (pq|rs) in chemist order, [M][M][M][M], with the
 *    8-fold permutational symmetry of real orbitals.
 *  - "device" pointers are HIP device memory of the context's device (torch
 *    tensors' data_ptr() work); "host" pointers are ordinary host memory.
 *  - The caller owns every input and output buffer.  The library owns the
 *    context, its cached string/link tables, plans, graphs and workspaces
 *    (hipMalloc'd, grown on demand, freed by mbefci_destroy).
 *  - hip_stream: the caller's stream (NULL = legacy default stream).  The
 *    library orders its own stream after all work already queued on it and
 *    makes it wait for the library's work before returning; calls that write
 *    host outputs return only when those outputs are valid.
 *  - Return value: MBEFCI_OK or a negative error code; on error no output is
 *    written and mbefci_last_error(ctx) describes the failure.  No C++
 *    exception crosses this boundary.
 *  - A CASCI here means: the lowest eigenvalue in the S_z sector with the
 *    given alpha/beta electron counts of the full-space Hamiltonian restricted
 *    to determinants whose frozen orbitals (reference-determinant occupied
 *    orbitals outside the active space) are doubly occupied and whose other
 *    inactive orbitals are empty.
 *  - Same inputs on the same device give bitwise identical outputs (fixed
 *    reduction orders, no floating-point atomics).
 */
#ifndef MBEFCI_H
#define MBEFCI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MBEFCI_OK = 0,
  MBEFCI_EINVAL = -1,      /* invalid argument (sizes, indices, symmetry, NaN) */
  MBEFCI_ENOMEM = -2,      /* device allocation failed or workspace cap exceeded */
  MBEFCI_ENOTCONV = -3,    /* a Davidson solve hit max_iter; see stats */
  MBEFCI_EDEVICE = -4,     /* HIP runtime error */
  MBEFCI_EUNSUPPORTED = -5 /* shape outside the compiled kernels (active n > 14) */
};

enum { MBEFCI_BATCHED = 0, MBEFCI_PER_LAUNCH = 1 };

typedef struct mbefci_ctx mbefci_ctx;

typedef struct {
  double conv_tol;       /* Davidson residual 2-norm tolerance (default 1e-6)       */
  int32_t max_iter;      /* Davidson iterations per CASCI (default 200)              */
  int32_t max_space;     /* subspace size before restart, 3..16 (default 5)         */
  int32_t nguess;        /* lowest-diagonal unit guess vectors, 1..8, below
                            max_space - 1 (default 1), for CASCIs that use
                            neither their whole space nor a P-space; every
                            solve also starts from one dense vector with
                            weight in every symmetry sector, orthogonalised
                            against the other guesses                       */
  int32_t mode;          /* MBEFCI_BATCHED (default) or MBEFCI_PER_LAUNCH            */
  int32_t use_graph;     /* batched mode: replay captured iterations (default 1)     */
  int32_t tile;          /* sigma tile width 32/64/128 (one alpha string per tile);
                            0 = autotuned schedule: the first batched solve of a
                            plan times the candidates per active size (also
                            flattened tiles of 32 or 64 consecutive
                            determinants for active sizes up to 9) and keeps
                            the fastest; a later candidate must be 3% faster
                            to replace an earlier one (default 0)             */
  int32_t keep_ci;       /* keep converged CI vectors for the backward (default 1)   */
  int32_t validate;      /* host checks of integral symmetry/finiteness (default 1)  */
  int32_t sigma_pass_mb; /* sigma sweeps run in passes whose G block (the W-contracted
                            pair array) stays below this many MiB, so that it is
                            re-read from the on-die cache and its memory is bounded;
                            0 = one pass (default 0) */
  int32_t precond;       /* Davidson correction: 0 = diagonal (theta - H_II)^-1 r
                            (with the P-space block below), where, when
                            conv_tol < 1e-7, a CASCI whose residual norm has
                            fallen below 1e-7 takes the Olsen form for the
                            rest of its solve; 1 = Olsen-corrected, orthogonal
                            to the Ritz vector, every iteration (default 0) */
  int32_t pspace;        /* largest P-space, 0..112: a CASCI of ndet > 112
                            determinants uses the P = min(pspace, ndet / 64)
                            determinants of lowest diagonal energy, whose block
                            H_PP is diagonalised once per CASCI; it gives the
                            guess and, on that block, the exact
                            (theta - H_PP)^-1 correction.  P < 24, or
                            pspace = 0: unit-vector guesses and the diagonal
                            correction only.  CASCIs of at most 112
                            determinants are always solved from their
                            whole-space block.  With precond = 1 the P-space
                            gives the guess only and every iteration takes
                            the Olsen correction (default 112)               */
  int32_t screen_batch;  /* most CASCIs per solve batch of mbefci_mbe_screened
                            (an order with more tuples, or more than 2^25
                            determinants, is solved in several batches);
                            0 = 65536 (default 0)                            */
  int64_t max_workspace; /* workspace cap in bytes, 0 = no cap                       */
  const char* tune_cache;/* autotuner cache file (read/written) or NULL: one line per
                            active size n, "n tile tiles_per_workgroup" (tile
                            -32 or -64: flattened tiles)                      */
} mbefci_opts;

typedef struct {
  int32_t norb;            /* M (1..64)                                              */
  const double* h1;        /* device [M*M], symmetric                                */
  const double* eri;       /* device [M^4], (pq|rs), 8-fold symmetric                */
  double e_const;          /* constant energy shift                                  */
  int32_t nocc;            /* number of doubly occupied orbitals of the reference    */
  const int32_t* occ;      /* host [nocc]: those orbitals (the set O)                */
  int32_t nref;            /* |R| (may be 0: the vacuum reference of Eq. 3)          */
  const int32_t* ref;      /* host [nref]: reference space R                         */
  int32_t nexp;            /* |X|                                                    */
  const int32_t* exp;      /* host [nexp]: expansion space X, disjoint from R        */
  int32_t max_order;       /* k, 0..nexp (0: only the reference CASCI)               */
  const int32_t* orbsym;   /* host [M] point-group irreps 0..7 of the MOs (D2h or a
                              subgroup, product = XOR), or NULL.  With irreps every
                              CASCI is solved in the totally symmetric irrep (that of
                              the closed-shell reference determinant) on the
                              point-group blocked path; supported by
                              mbefci_mbe_screened only (EUNSUPPORTED elsewhere)     */
} mbefci_problem;

typedef struct {
  int64_t ntuples;           /* CASCIs solved, the reference CASCI included       */
  int64_t nsingle;           /* of which single-determinant (no eigen-solve)      */
  int64_t sigma_calls;       /* sigma = Hc evaluations summed over CASCIs         */
  int64_t ndet_total;        /* sum of determinant counts                         */
  int32_t max_iters;         /* largest Davidson iteration count                  */
  int32_t first_failed;      /* first CASCI index that did not converge, or -1    */
  int32_t nbuckets;          /* shape buckets                                     */
  int32_t graph_launches;    /* replays of the captured iteration graph           */
  double ms_total;           /* wall time of the call (host clock)                */
  double ms_solve;           /* device time of the Davidson phase (HIP events)    */
  double ms_tune;            /* host time spent autotuning so far on this context */
} mbefci_stats;

/* ---- context ------------------------------------------------------------ */
void mbefci_default_opts(mbefci_opts* opts);
/* Create a context on HIP device `device`.  opts == NULL takes the defaults. */
int mbefci_create(int device, const mbefci_opts* opts, mbefci_ctx** out);
void mbefci_destroy(mbefci_ctx* ctx);
/* Message of the last failure on ctx (valid until the next call on ctx). */
const char* mbefci_last_error(const mbefci_ctx* ctx);
/* New options apply from the next call.  Changing max_space, tile,
 * sigma_pass_mb, precond or pspace drops the cached plan (a backward then needs
 * a new forward); changing conv_tol or max_iter keeps the plan and captures its
 * iteration graph again.  A call that fails while building a plan leaves no
 * plan behind. */
int mbefci_set_opts(mbefci_ctx* ctx, const mbefci_opts* opts);
/* Workspace allocator (the context's arenas: Davidson vectors, sigma
 * intermediates, kept CI vectors, per-CASCI state): alloc(bytes, user) returns
 * device memory of the context's device, aligned to at least 256 bytes, or NULL
 * (the call that needed it then fails with ENOMEM); release(ptr, user) takes
 * back a block, called only after the library stream has finished every queued
 * use of it.  Both NULL: hipMalloc/hipFree (the default).  The small string and
 * link tables always come from hipMalloc.  Setting or clearing the allocator
 * releases every arena through the function that allocated it and drops the
 * cached plan (a backward must follow a new forward).  The callbacks run on the
 * thread that calls the library.  EINVAL: null ctx, or only one function. */
int mbefci_set_allocator(mbefci_ctx* ctx, void* (*alloc)(size_t bytes, void* user),
                         void (*release)(void* ptr, void* user), void* user);

/* ---- integer layer: strings and single-excitation link tables ------------
 * Every CASCI of the expansion (the constituent CASCI calculations whose
 * energies enter eps_T of Eq. 2) is a full CI in its active space, over the
 * determinants |Ia Ib> of an alpha and a beta string.  A string of nelec
 * electrons in norb active orbitals is a bitmask; strings are numbered in
 * ascending integer order (address = sum_j C(o_j, j) over the occupied
 * orbitals o_1 < o_2 < ..., the combinatorial number system).  The
 * determinant of alpha string Ia and beta string Ib has address
 * Ia * N_beta + Ib. */
int64_t mbefci_num_strings(int32_t norb, int32_t nelec);     /* C(norb, nelec); 0 if invalid */
int32_t mbefci_num_links(int32_t norb, int32_t nelec);       /* nelec*(norb-nelec+1)        */
/* Host, no context, no device: out host [nstr] uint64 bitmasks, ascending
 * (the caller allocates mbefci_num_strings(norb, nelec) entries).  EINVAL for
 * norb outside 0..64, nelec outside 0..norb, a null out, or more than 2^31 - 1
 * strings; ENOMEM if host memory runs out. */
int mbefci_strings(int32_t norb, int32_t nelec, uint64_t* out);
/* Host, no context, no device: out host [nstr][nlink][4] int32 = (p, q, J,
 * sign) with E_pq|I> = sign|J>, E_pq = a+_p a_q of one spin.  Per string: the
 * diagonal entries (o,o,I,+1) for occupied o ascending, then for occupied q
 * ascending and empty p ascending; sign = (-1)^(occupied orbitals strictly
 * between p and q), the parity of a+_p a_q on the occupation-number vector.
 * EINVAL for norb outside 0..32, nelec outside 0..norb or a null out. */
int mbefci_link_table(int32_t norb, int32_t nelec, int32_t* out);
/* The same two tables built by the library's kernels into device memory of
 * ctx's device (out: device [nstr] / [nstr][nlink][4]), on hip_stream. */
int mbefci_strings_device(mbefci_ctx* ctx, int32_t norb, int32_t nelec, uint64_t* out,
                          void* hip_stream);
int mbefci_link_table_device(mbefci_ctx* ctx, int32_t norb, int32_t nelec, int32_t* out,
                             void* hip_stream);
/* Number of tuples of 1..max_order orbitals out of nexp: sum_n C(nexp, n),
 * the CASCIs behind the order sums E^(1..max_order) of Eq. 1 (order n holds
 * the C(nexp, n) increments of Eq. 2).  0 for invalid arguments. */
int64_t mbefci_num_tuples(int32_t nexp, int32_t max_order);

/* ---- one CASCI Hamiltonian in an active space ---------------------------
 * The Hamiltonian whose lowest eigenvalue is a CASCI energy of Eq. 1 / Eq. 2,
 * H = sum h_pq E_pq + 1/2 sum (pq|rs) (E_pq E_rs - delta_qr E_ps) + e_core,
 * on the determinants of the active space.  h1 device [n*n], eri device
 * [n^4] (active-space integrals), e_core the constant added to every
 * diagonal element.  Determinant layout [Na][Nb].  The sigma build is the
 * string-driven Knowles-Handy / Olsen factorisation (the paper leaves the
 * CASCI solver to its host program; this is the solver's own method). */
/* diag: device [Na*Nb], H_II including e_core. */
int mbefci_hdiag(mbefci_ctx* ctx, int32_t norb, int32_t nalpha, int32_t nbeta, const double* h1,
                 const double* eri, double e_core, double* diag, void* hip_stream);
/* sigma = H c (e_core included): c, sigma device [Na*Nb]. */
int mbefci_sigma(mbefci_ctx* ctx, int32_t norb, int32_t nalpha, int32_t nbeta, const double* h1,
                 const double* eri, double e_core, const double* c, double* sigma,
                 void* hip_stream);

/* sigma = H c as mbefci_sigma computes it, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Allocates nothing: every intermediate (string, link
 * and pair tables, W, the contracted pair array G, work lists) lives in one
 * static device array of 32 MiB per GPU, held until the process ends.  Runs
 * only kernel launches, on hip_stream itself (no library stream, no events,
 * no synchronisation, no host copies, no memset nodes), so it may be captured
 * into a graph.  The integrals are not validated on the host (opts.validate
 * does not apply).  Shapes: norb 0..14 whose tables, W and G fit the 32 MiB
 * (every shape up to CAS(10,10), 28.8 MB at 5+5 electrons); larger ones
 * return ENOMEM with the size in mbefci_last_error(ctx).  ctx supplies the
 * device and the error message only: neither its plan nor its workspaces are
 * touched, so its other calls are unaffected.  Every call on a GPU shares that
 * GPU's array and leaves its contents behind: calls that overlap on one GPU
 * (several streams, threads or contexts) race and must be serialised by the
 * caller.  c and sigma: device [Na*Nb], distinct. */
int mbefci_sigma_noalloc(mbefci_ctx* ctx, int32_t norb, int32_t nalpha, int32_t nbeta,
                         const double* h1, const double* eri, double e_core, const double* c,
                         double* sigma, void* hip_stream);

/* ---- CASCI solves ---------------------------------------------------------
 * A CASCI energy is the lowest eigenvalue of H above (the constituent CASCI
 * calculations of Eq. 1; eps_T of Eq. 2 is the energy of the CASCI in
 * R u T minus E_ref), found by a Davidson solve to opts.conv_tol.
 *
 * One CASCI: integrals h1 device [n*n], eri device [n^4], e_core; e_out host
 * [1] the energy; ci_out device [Na*Nb] the normalised eigenvector, rdm1
 * device [n*n] gamma_pq = <E_pq>, rdm2 device [n^4]
 * Gamma_pqrs = <E_pq E_rs> - delta_qr gamma_ps symmetrised over the eight
 * index permutations of (pq|rs) (the gradient convention: dE/dh = gamma,
 * dE/d(pq|rs) = Gamma/2 for symmetric perturbations), each NULL if not
 * wanted.  EINVAL if any of them is asked for with keep_ci = 0. */
int mbefci_casci(mbefci_ctx* ctx, int32_t norb, int32_t nalpha, int32_t nbeta, const double* h1,
                 const double* eri, double e_core, double* e_out, double* ci_out, double* rdm1,
                 double* rdm2, void* hip_stream);
/* A batch of nprob independent CASCIs of one shape, solved together (one
 * Davidson iteration advances all of them): h1s[i] device [n*n], eris[i]
 * device [n^4] (host arrays of device pointers), e_core host [nprob].
 * e_out host [nprob]: lowest eigenvalues.  ci_out: NULL or host array of
 * nprob device pointers [Na*Nb] (entries may be NULL) receiving the
 * normalised eigenvectors (EINVAL with keep_ci = 0). */
int mbefci_casci_batch(mbefci_ctx* ctx, int32_t nprob, int32_t norb, int32_t nalpha,
                       int32_t nbeta, const double* const* h1s, const double* const* eris,
                       const double* e_core, double* e_out, double* const* ci_out,
                       mbefci_stats* stats, void* hip_stream);
/* RDMs (as for mbefci_casci) of the CI vectors kept by the last CASCI solve
 * on ctx (mbefci_casci_batch or mbefci_casci): rdm1s[i] device [n*n],
 * rdm2s[i] device [n^4]; either array may be NULL. */
int mbefci_casci_rdm(mbefci_ctx* ctx, double* const* rdm1s, double* const* rdm2s,
                     void* hip_stream);

/* ---- point-group blocked CASCIs ---------------------------------------------
 * The paper's Cr2 expansion solves its CASCIs with D2h symmetry (Fig. 3
 * discussion: the largest, 2.07e7 determinants "with D2h symmetry").  Orbital
 * irreps of D2h or a subgroup are labels 0..7 whose product is their XOR; a
 * string's irrep is the XOR of its occupied orbitals' labels, a determinant's
 * the XOR of its two strings'.  A CASCI of irrep G holds only the determinants
 * of irrep G.  Layout of its CI vector: the strings of each spin sorted by
 * (irrep, bitmask); blocks over the alpha irreps a = 0..7 in order, block a =
 * [alpha strings of irrep a][beta strings of irrep a^G] row-major.  Sigma runs
 * one FP64-MFMA contraction per pair class s (pairs p >= q with irr(p)^irr(q)
 * = s) on the determinants of irrep G^s.  RDMs are not available for these
 * CASCIs (mbefci_casci_rdm returns EUNSUPPORTED). */
/* Host, no context: determinants of irrep wfnsym of norb orbitals with
 * irreps orbsym [norb] (0..7) and nalpha / nbeta electrons; EINVAL (negative)
 * for invalid arguments. */
int64_t mbefci_sym_ndet(int32_t norb, int32_t nalpha, int32_t nbeta, const int32_t* orbsym,
                        int32_t wfnsym);
/* A batch of same-shape CASCIs in irrep wfnsym (as mbefci_casci_batch; orbsym
 * host [norb] irreps of the active orbitals).  ci_out[i]: device
 * [mbefci_sym_ndet(...)] in the layout above.  EINVAL when the irrep has no
 * determinant. */
int mbefci_casci_sym(mbefci_ctx* ctx, int32_t nprob, int32_t norb, int32_t nalpha,
                     int32_t nbeta, const int32_t* orbsym, int32_t wfnsym,
                     const double* const* h1s, const double* const* eris, const double* e_core,
                     double* e_out, double* const* ci_out, mbefci_stats* stats,
                     void* hip_stream);
/* sigma = H c (e_core included) on the determinants of irrep wfnsym: c, sigma
 * device [mbefci_sym_ndet(...)] in the layout above. */
int mbefci_sigma_sym(mbefci_ctx* ctx, int32_t norb, int32_t nalpha, int32_t nbeta,
                     const int32_t* orbsym, int32_t wfnsym, const double* h1, const double* eri,
                     double e_core, const double* c, double* sigma, void* hip_stream);

/* ---- many-body expansion -------------------------------------------------
 * Solves E_ref (CASCI of R) and the CASCI of R u T for every tuple T of
 * 1..max_order expansion orbitals, then forms the increments of Eq. 2 and the
 * order sums of Eq. 1.  Outputs (host): e_ref, e_order [max_order],
 * e_total = e_ref + sum e_order, tuple_incr [num_tuples] or NULL (order by
 * order, lexicographic tuples of the sorted X within an order) and
 * tuple_energy [num_tuples] or NULL (the CASCI energies E(R u T), same order).  Converged
 * CI vectors are kept on ctx for mbefci_mbe_backward when keep_ci is set.
 * Every CASCI is solved in one batch (Davidson subspace, sigma intermediates
 * and kept CI vectors of all tuples at once); an expansion too large for the
 * device gives ENOMEM.  mbefci_mbe_screened with t_init = 0 computes the same
 * energies order by order in bounded batches (no backward). */
int mbefci_mbe_forward(mbefci_ctx* ctx, const mbefci_problem* prob, double* e_ref,
                       double* e_order, double* e_total, double* tuple_incr,
                       double* tuple_energy, mbefci_stats* stats, void* hip_stream);
/* Gradient of L = g[0] E_ref + sum_n g[n] E^(n) (g host [1+max_order]) of the
 * last forward on ctx with respect to the MO integrals: d_h1 device [M*M]
 * (symmetric) and d_eri device [M^4] (8-fold symmetrised); both overwritten. */
int mbefci_mbe_backward(mbefci_ctx* ctx, const double* grad_out, double* d_h1, double* d_eri,
                        void* hip_stream);

/* ---- partitions -------------------------------------------------------------
 * The paper's three partitions of the M orbitals into a reference space R
 * and an expansion space X (the discussion before Eq. 3), given the occupied
 * orbitals O of the reference determinant:
 *   MBEFCI_TYPE1: X = O (expansion over occupied MOs), R = the virtual MOs;
 *   MBEFCI_TYPE2: R = O, X = the virtual MOs;
 *   MBEFCI_TYPE3: R empty (vacuum reference), X = all M orbitals.
 * Host only, no ctx.  ref / exp: host [M] buffers; *nref, *nexp receive the
 * sizes; both lists ascending.  EINVAL for an unknown type, M outside 1..64 or
 * a bad occupied list. */
enum { MBEFCI_TYPE1 = 1, MBEFCI_TYPE2 = 2, MBEFCI_TYPE3 = 3 };
int mbefci_partition(int32_t type, int32_t norb, int32_t nocc, const int32_t* occ, int32_t* ref,
                     int32_t* nref, int32_t* exp, int32_t* nexp);

/* ---- screened expansion ---------------------------------------------------
 * The order-by-order driver of the paper's production runs (the tuple
 * screening described with Eq. 4).  Order 1 holds every expansion orbital.
 * Spawning is per parent: a computed tuple P of order k and a candidate
 * orbital c of X outside P spawn P + c when, for some (k-1)-subtuple S of P,
 * the tuple S + c was computed with |Delta eps_{S+c}| > T_tup(S + c) (a tuple
 * never computed has no increment and spawns nothing; P itself is not tested).
 * Order k+1 is the union over all parents and candidates.  Here (Eq. 4)
 *   T_tup = 0                                 if M_tup <  m_init,
 *   T_tup = t_init * a^(M_tup - m_init)       otherwise,
 * and M_tup = max(occupied MOs, virtual MOs) of the tested tuple.  With an
 * empty reference space (Eq. 3) tuples of only occupied or only virtual MOs
 * have vanishing increments by construction: they are not computed (and are
 * no parents), and every mixed pair is (order 2 is the first order).  Increments follow Eq. 2 over the computed
 * sub-tuples (a sub-tuple never computed contributes 0).  Outputs (host):
 * e_ref, e_order [max_order] (0 for orders with no tuple), e_total,
 * n_order [max_order] (tuples computed per order).  The computed tuples and
 * their increments stay on ctx for mbefci_screened_tuples; the call drops the
 * cached plan of mbefci_mbe_forward (no backward follows a screened call).
 * Each order is solved in batches of at most opts.screen_batch CASCIs and
 * 2^25 determinants, so device memory bounds the batch, not the expansion.
 * Errors: EINVAL for t_init < 0, a < 1, m_init < 0 or a bad problem. */
typedef struct {
  double t_init;          /* T_init in E_h (the paper: 1e-10)                         */
  double a;               /* relaxation factor a >= 1 (the paper: 5.0, or 2.5)        */
  int32_t m_init;         /* M_init (the paper: 3)                                    */
  int32_t pad_;
} mbefci_screen;
int mbefci_mbe_screened(mbefci_ctx* ctx, const mbefci_problem* prob, const mbefci_screen* scr,
                        double* e_ref, double* e_order, double* e_total, int64_t* n_order,
                        mbefci_stats* stats, void* hip_stream);
/* The tuples computed at `order` (1..max_order) by the last screened call on
 * ctx, in lexicographic order of the sorted orbital lists: tuples host
 * [count][order] orbital indices (or NULL), increments host [count] Delta eps
 * (or NULL).  Returns count, or a negative error code. */
int64_t mbefci_screened_tuples(mbefci_ctx* ctx, int32_t order, int32_t* tuples,
                               double* increments);

/* ---- measurement ----------------------------------------------------------
 * Re-times the sigma = Hc kernels of the last mbefci_casci / mbefci_mbe_forward
 * on ctx: each kernel of one sigma sweep over the whole batch is replayed
 * `reps` times between HIP events on the library stream (the stream the
 * kernels run on).  Replays recompute identical values; the results of the
 * last call are unchanged.  Fills up to `cap` records, *count = records. */
typedef struct {
  char name[64];          /* kernel and shape, e.g. "sigma_dgemm<n=10,tile=64>",
                             "sigma_dgemm_flat<n=8,tile=32>", "sigma_gather"        */
  int32_t launches;       /* launches of this kernel in one sigma sweep               */
  int32_t pad_;
  double ms_per_launch;   /* average device time of one launch                        */
  double flops;           /* algorithmic flops of one launch (average)                */
  double bytes;           /* algorithmic HBM bytes of one launch (average)            */
  double ndet;            /* determinants processed by one launch (average)           */
} mbefci_kernel_time;
int mbefci_time_kernels(mbefci_ctx* ctx, int32_t reps, mbefci_kernel_time* out, int32_t cap,
                        int32_t* count);
/* The device's attainable peaks, measured on ctx's device and stream:
 * *fp64_mfma_tflops from eight independent chains of v_mfma_f64_16x16x4f64
 * per wave issued from registers (16 blocks of 256 threads per CU, best of
 * three launches), *copy_gbps from
 * a 16-byte-vector copy of 256 MiB (bytes read plus written, best of five).
 * They put the roofline fractions beside the published peaks (78.6 TFLOP/s
 * FP64 matrix, 8 TB/s HBM).  Uses a 512 MiB workspace that the context
 * keeps until it is destroyed.  Errors: EINVAL (null output), EDEVICE. */
int mbefci_probe_peaks(mbefci_ctx* ctx, double* fp64_mfma_tflops, double* copy_gbps);

#ifdef __cplusplus
}
#endif
#endif /* MBEFCI_H */
