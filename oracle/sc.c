/*
 * Oracle core (TEST INFRASTRUCTURE ONLY -- never linked by the product path).
 *
 * Plain Slater-Condon rules over full-space determinants, written from the
 * textbook second-quantised Hamiltonian
 *
 *   H = sum_{PQ} [P|Q] a+_P a_Q + 1/2 sum_{PQRS} [PQ|RS] a+_P a+_R a_S a_Q
 *
 * over spin orbitals P = (p, sigma), with [PQ|RS] = (pq|rs) when
 * sigma_P = sigma_Q and sigma_R = sigma_S, else 0.  This is the Hamiltonian
 * every CASCI of the many-body expansion diagonalises (the expansion of
 * Eq. 1 / Eq. 2 is over the energies of such CASCI problems).
 *
 * A determinant is an occupation-number vector of 2M spin orbitals, stored as
 * two uint64 masks (alpha, beta) over the M spatial orbitals; spin-orbital
 * index = sigma*M + p (all alpha before all beta), and a determinant is the
 * product of creation operators in ascending spin-orbital order acting on the
 * vacuum.  Creation/annihilation act with the sign (-1)^(number of occupied
 * spin orbitals of lower index): the textbook occupation-number definition.
 *
 * No blocking, factorisation or string-driven tricks: every matrix element is
 * evaluated from the rules directly.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t m[2]; /* m[0] alpha, m[1] beta */
} det_t;

static inline int popc(uint64_t x) { return __builtin_popcountll(x); }

/* number of occupied spin orbitals with index < P (P = sigma*M + p) */
static int count_below(const det_t* d, int sigma, int p) {
    uint64_t below = (p == 0) ? 0 : (((uint64_t)1 << p) - 1);
    int n = popc(d->m[sigma] & below);
    if (sigma == 1) n += popc(d->m[0]);
    return n;
}

/* a_P on d: returns sign (+1/-1) or 0 when P is empty */
static int annihilate(det_t* d, int sigma, int p) {
    uint64_t bit = (uint64_t)1 << p;
    if (!(d->m[sigma] & bit)) return 0;
    int s = (count_below(d, sigma, p) & 1) ? -1 : 1;
    d->m[sigma] &= ~bit;
    return s;
}

/* a+_P on d: returns sign or 0 when P is occupied */
static int create(det_t* d, int sigma, int p) {
    uint64_t bit = (uint64_t)1 << p;
    if (d->m[sigma] & bit) return 0;
    int s = (count_below(d, sigma, p) & 1) ? -1 : 1;
    d->m[sigma] |= bit;
    return s;
}

/* spin-orbital one- and two-electron integrals */
static inline double so_h(const double* h, int M, int P, int Q) {
    if (P / M != Q / M) return 0.0;
    return h[(P % M) * M + (Q % M)];
}
static inline double so_g(const double* g, int M, int P, int Q, int R, int S) {
    if (P / M != Q / M || R / M != S / M) return 0.0;
    int p = P % M, q = Q % M, r = R % M, s = S % M;
    return g[(((size_t)p * M + q) * M + r) * M + s];
}

/* list occupied spin orbitals of d (ascending); returns count */
static int occupied(const det_t* d, int M, int* out) {
    int n = 0;
    for (int sigma = 0; sigma < 2; ++sigma)
        for (int p = 0; p < M; ++p)
            if (d->m[sigma] >> p & 1) out[n++] = sigma * M + p;
    return n;
}

/*
 * <I|H|J> (without the constant shift) for determinants I, J.
 * Slater-Condon rules: identical, single and double differences; zero beyond.
 */
double sc_element(int M, const double* h, const double* g,
                  uint64_t ia, uint64_t ib, uint64_t ja, uint64_t jb) {
    det_t I = {{ia, ib}}, J = {{ja, jb}};
    int diff = popc(ia ^ ja) + popc(ib ^ jb);
    if (diff > 4) return 0.0;
    if (popc(ia) + popc(ib) != popc(ja) + popc(jb)) return 0.0;
    int occ[128];
    if (diff == 0) {
        int n = occupied(&I, M, occ);
        double e = 0.0;
        for (int x = 0; x < n; ++x) e += so_h(h, M, occ[x], occ[x]);
        for (int x = 0; x < n; ++x)
            for (int y = 0; y < n; ++y)
                e += 0.5 * (so_g(g, M, occ[x], occ[x], occ[y], occ[y]) -
                            so_g(g, M, occ[x], occ[y], occ[y], occ[x]));
        return e;
    }
    /* holes: occupied in J, empty in I ; particles: occupied in I, empty in J.
       We evaluate <I| a+_a a+_b a_j a_i |J> style excitations from J to I. */
    int holes[2], parts[2], nh = 0, np_ = 0;
    for (int sigma = 0; sigma < 2; ++sigma)
        for (int p = 0; p < M; ++p) {
            int inI = (int)(I.m[sigma] >> p & 1), inJ = (int)(J.m[sigma] >> p & 1);
            if (inJ && !inI) holes[nh++] = sigma * M + p;
            if (inI && !inJ) parts[np_++] = sigma * M + p;
        }
    if (diff == 2) {
        int i = holes[0], a = parts[0];
        det_t t = J;
        int s = annihilate(&t, i / M, i % M);
        s *= create(&t, a / M, a % M);
        /* t == I by construction */
        int n = occupied(&J, M, occ);
        double e = so_h(h, M, a, i);
        for (int x = 0; x < n; ++x) {
            int k = occ[x];
            e += so_g(g, M, a, i, k, k) - so_g(g, M, a, k, k, i);
        }
        return s * e;
    }
    /* diff == 4: double excitation J -> I : I = a+_a a+_b a_j a_i J */
    int i = holes[0], j = holes[1], a = parts[0], b = parts[1];
    det_t t = J;
    int s = annihilate(&t, i / M, i % M);
    s *= annihilate(&t, j / M, j % M);
    s *= create(&t, b / M, b % M);
    s *= create(&t, a / M, a % M);
    return s * (so_g(g, M, a, i, b, j) - so_g(g, M, a, j, b, i));
}

/* neighbour lists of a string set: for each string, strings that differ by
   at most two electrons, with the number of differing electrons */
typedef struct {
    int64_t* start; /* [n+1] */
    int32_t* idx;
    int8_t* deg;
} nbr_t;

static nbr_t neighbours(int n, const uint64_t* s) {
    nbr_t r;
    r.start = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
    int64_t cnt = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (popc(s[i] ^ s[j]) <= 4) ++cnt;
    r.idx = (int32_t*)malloc(sizeof(int32_t) * (cnt ? cnt : 1));
    r.deg = (int8_t*)malloc(cnt ? cnt : 1);
    cnt = 0;
    for (int i = 0; i < n; ++i) {
        r.start[i] = cnt;
        for (int j = 0; j < n; ++j) {
            int d = popc(s[i] ^ s[j]);
            if (d <= 4) {
                r.idx[cnt] = j;
                r.deg[cnt] = (int8_t)(d / 2);
                ++cnt;
            }
        }
    }
    r.start[n] = cnt;
    return r;
}

static void free_nbr(nbr_t* r) {
    free(r->start);
    free(r->idx);
    free(r->deg);
}

/*
 * Sparse H over the product space {(alpha[i], beta[j])}, determinant index
 * i*nb + j.  Pass indices == NULL to only count the non-zeros (returned).
 * Rows are written in increasing column order.
 */
int64_t sc_build_csr(int M, const double* h, const double* g, double ecore,
                     int na, const uint64_t* amask, int nb, const uint64_t* bmask,
                     int64_t* indptr, int32_t* indices, double* data) {
    nbr_t A = neighbours(na, amask), B = neighbours(nb, bmask);
    int64_t nnz = 0;
    for (int ia = 0; ia < na; ++ia)
        for (int ib = 0; ib < nb; ++ib) {
            int64_t row = (int64_t)ia * nb + ib;
            if (indptr) indptr[row] = nnz;
            for (int64_t x = A.start[ia]; x < A.start[ia + 1]; ++x) {
                int ja = A.idx[x], da = A.deg[x];
                for (int64_t y = B.start[ib]; y < B.start[ib + 1]; ++y) {
                    int jb = B.idx[y], db = B.deg[y];
                    if (da + db > 2) continue;
                    if (indices) {
                        double v = sc_element(M, h, g, amask[ia], bmask[ib], amask[ja], bmask[jb]);
                        if (da + db == 0) v += ecore;
                        indices[nnz] = (int32_t)((int64_t)ja * nb + jb);
                        data[nnz] = v;
                    }
                    ++nnz;
                }
            }
        }
    if (indptr) indptr[(int64_t)na * nb] = nnz;
    free_nbr(&A);
    free_nbr(&B);
    return nnz;
}

/* diagonal of H over the product space */
void sc_diagonal(int M, const double* h, const double* g, double ecore,
                 int na, const uint64_t* amask, int nb, const uint64_t* bmask, double* out) {
    for (int ia = 0; ia < na; ++ia)
        for (int ib = 0; ib < nb; ++ib)
            out[(int64_t)ia * nb + ib] =
                ecore + sc_element(M, h, g, amask[ia], bmask[ib], amask[ia], bmask[ib]);
}

/*
 * sigma_I = sum_J <I|H|J> c_J for a list of sampled rows I (product-space
 * indices), without forming H.  Every J of the product space within two
 * electrons of I is visited.
 */
void sc_sigma_rows(int M, const double* h, const double* g, double ecore,
                   int na, const uint64_t* amask, int nb, const uint64_t* bmask,
                   const double* c, int nrows, const int64_t* rows, double* out) {
    for (int r = 0; r < nrows; ++r) {
        int64_t I = rows[r];
        int ia = (int)(I / nb), ib = (int)(I % nb);
        double acc = 0.0;
        for (int ja = 0; ja < na; ++ja) {
            int da = popc(amask[ia] ^ amask[ja]);
            if (da > 4) continue;
            for (int jb = 0; jb < nb; ++jb) {
                int db = popc(bmask[ib] ^ bmask[jb]);
                if (da + db > 4) continue;
                double v = sc_element(M, h, g, amask[ia], bmask[ib], amask[ja], bmask[jb]);
                if (da + db == 0) v += ecore;
                acc += v * c[(int64_t)ja * nb + jb];
            }
        }
        out[r] = acc;
    }
}

static int find_u64(int n, const uint64_t* s, uint64_t key) {
    int lo = 0, hi = n - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (s[mid] == key) return mid;
        if (s[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/*
 * Spin-summed reduced density matrices of a real vector c over the product
 * space, in the full M-orbital space:
 *   gamma[p,q]     = sum_sigma <c| a+_{p sigma} a_{q sigma} |c>
 *   Gamma[p,q,r,s] = sum_{sigma,tau} <c| a+_{p sigma} a+_{r tau} a_{s tau} a_{q sigma} |c>
 * (Gamma = <E_pq E_rs> - delta_qr gamma_ps).  Every operator string is applied
 * to every determinant J; the result is looked up in the product space (a
 * determinant outside it has zero coefficient).  gamma [M*M], Gamma [M^4] are
 * overwritten.
 */
void sc_rdm12(int M, int na, const uint64_t* amask, int nb, const uint64_t* bmask,
              const double* c, double* gamma, double* Gamma) {
    memset(gamma, 0, sizeof(double) * M * M);
    memset(Gamma, 0, sizeof(double) * (size_t)M * M * M * M);
    for (int ja = 0; ja < na; ++ja)
        for (int jb = 0; jb < nb; ++jb) {
            double cj = c[(int64_t)ja * nb + jb];
            if (cj == 0.0) continue;
            det_t J = {{amask[ja], bmask[jb]}};
            for (int sq = 0; sq < 2; ++sq)
                for (int q = 0; q < M; ++q) {
                    det_t t1 = J;
                    int s1 = annihilate(&t1, sq, q);
                    if (!s1) continue;
                    /* one-body: a+_p a_q, p of the same spin */
                    for (int p = 0; p < M; ++p) {
                        det_t t = t1;
                        int s = s1 * create(&t, sq, p);
                        if (!s) continue;
                        int ia = find_u64(na, amask, t.m[0]);
                        int ib = find_u64(nb, bmask, t.m[1]);
                        if (ia < 0 || ib < 0) continue;
                        gamma[p * M + q] += s * c[(int64_t)ia * nb + ib] * cj;
                    }
                    /* two-body: a+_p a+_r a_s a_q */
                    for (int ss = 0; ss < 2; ++ss)
                        for (int s_ = 0; s_ < M; ++s_) {
                            det_t t2 = t1;
                            int s2 = s1 * annihilate(&t2, ss, s_);
                            if (!s2) continue;
                            for (int r = 0; r < M; ++r) {
                                det_t t3 = t2;
                                int s3 = s2 * create(&t3, ss, r);
                                if (!s3) continue;
                                for (int p = 0; p < M; ++p) {
                                    det_t t4 = t3;
                                    int s4 = s3 * create(&t4, sq, p);
                                    if (!s4) continue;
                                    int ia = find_u64(na, amask, t4.m[0]);
                                    int ib = find_u64(nb, bmask, t4.m[1]);
                                    if (ia < 0 || ib < 0) continue;
                                    Gamma[(((size_t)p * M + q) * M + r) * M + s_] +=
                                        s4 * c[(int64_t)ia * nb + ib] * cj;
                                }
                            }
                        }
                }
        }
}

/*
 * Matrix-free sigma = H c over the product space {(alpha[i], beta[j])} for
 * spaces too large for a stored H (CAS(14,14): 11.8 M determinants).  Row I
 * visits only the determinants J within two electrons of I, reached by
 * exciting one spin string (singles and same-spin doubles) or both strings
 * once (opposite-spin doubles); every element is a Slater-Condon element:
 *
 *  - a same-spin double, and the one-spin part of a same-spin single, are
 *    sc_element of the two strings with the other spin empty.  In the
 *    alpha-first ordering a beta operator passes every alpha electron and an
 *    alpha operator none of the beta ones, and an excitation has an even
 *    number of operators, so the sign never depends on the other string; a
 *    double's value does not either, and for a single the other spin adds
 *    only its Coulomb term sgn * sum_{k in other} (ai|kk) (the exchange
 *    integral between different spins vanishes);
 *  - an opposite-spin double (alpha i->a, beta j->b) is
 *    sgn_alpha * sgn_beta * (ai|bj), the sign of each single excitation
 *    taken on its own string (the product of the four operator signs of the
 *    textbook rule reduces to this, the alpha electrons being counted twice
 *    by the beta operators);
 *  - the diagonal is passed in (sc_diagonal).
 *
 * These reductions are pinned against sc_build_csr on small spaces.  Setup
 * builds per-string excitation lists (strings outside the space, e.g. with a
 * frozen orbital emptied or a deleted one filled, are skipped); sigma rows
 * are computed for alpha strings [ia_lo, ia_hi), so callers can split the
 * rows over threads.
 */
typedef struct {
    int32_t t;      /* index of the excited string */
    int8_t a, i;    /* created, annihilated orbital */
    int8_t sgn;     /* sign of a+_a a_i on the source string */
    double v1;      /* sc_element of the one-spin part (other spin empty) */
} sc_single_t;

typedef struct {
    int32_t t;
    double v;
} sc_double_t;

typedef struct {
    int M, n;
    const double* g;
    int ns;              /* singles per string (max) */
    int nd;              /* doubles per string (max) */
    int32_t* ns_of;      /* [n] singles of string s */
    int32_t* nd_of;      /* [n] */
    sc_single_t* sing;   /* [n][ns] */
    sc_double_t* dbl;    /* [n][nd] */
    double* coul;        /* [n][M*M]: sum_{k in s} (ai|kk) */
} sc_spin_t;

typedef struct {
    int M, na, nb;
    const double* diag;
    sc_spin_t A, B;
} sc_direct_t;

static int spin_setup(sc_spin_t* T, int M, const double* h, const double* g, int n,
                      const uint64_t* s, int spin) {
    T->M = M;
    T->n = n;
    T->g = g;
    int ne = n ? popc(s[0]) : 0;
    T->ns = ne * (M - ne) + 1;
    T->nd = (ne * (ne - 1) / 2) * ((M - ne) * (M - ne - 1) / 2) + 1;
    T->ns_of = (int32_t*)calloc(n ? n : 1, sizeof(int32_t));
    T->nd_of = (int32_t*)calloc(n ? n : 1, sizeof(int32_t));
    T->sing = (sc_single_t*)malloc(sizeof(sc_single_t) * (size_t)(n ? n : 1) * T->ns);
    T->dbl = (sc_double_t*)malloc(sizeof(sc_double_t) * (size_t)(n ? n : 1) * T->nd);
    T->coul = (double*)calloc((size_t)(n ? n : 1) * M * M, sizeof(double));
    if (!T->ns_of || !T->nd_of || !T->sing || !T->dbl || !T->coul) return -1;
    for (int x = 0; x < n; ++x) {
        uint64_t m = s[x];
        double* cl = T->coul + (size_t)x * M * M;
        for (int a = 0; a < M; ++a)
            for (int i = 0; i < M; ++i) {
                double acc = 0.0;
                for (int k = 0; k < M; ++k)
                    if (m >> k & 1) acc += g[(((size_t)a * M + i) * M + k) * M + k];
                cl[a * M + i] = acc;
            }
        sc_single_t* S1 = T->sing + (size_t)x * T->ns;
        sc_double_t* S2 = T->dbl + (size_t)x * T->nd;
        int c1 = 0, c2 = 0;
        for (int i = 0; i < M; ++i) {
            if (!(m >> i & 1)) continue;
            for (int a = 0; a < M; ++a) {
                if (m >> a & 1) continue;
                uint64_t t = (m & ~((uint64_t)1 << i)) | ((uint64_t)1 << a);
                int ti = find_u64(n, s, t);
                if (ti < 0) continue;
                det_t d = {{m, 0}};
                int sg = annihilate(&d, 0, i);
                sg *= create(&d, 0, a);
                double v1 = spin == 0 ? sc_element(M, h, g, t, 0, m, 0)
                                      : sc_element(M, h, g, 0, t, 0, m);
                S1[c1].t = ti;
                S1[c1].a = (int8_t)a;
                S1[c1].i = (int8_t)i;
                S1[c1].sgn = (int8_t)sg;
                S1[c1].v1 = v1;
                ++c1;
            }
        }
        for (int i = 0; i < M; ++i) {
            if (!(m >> i & 1)) continue;
            for (int j = i + 1; j < M; ++j) {
                if (!(m >> j & 1)) continue;
                for (int a = 0; a < M; ++a) {
                    if (m >> a & 1) continue;
                    for (int b = a + 1; b < M; ++b) {
                        if (m >> b & 1) continue;
                        uint64_t t = (m & ~(((uint64_t)1 << i) | ((uint64_t)1 << j))) |
                                     ((uint64_t)1 << a) | ((uint64_t)1 << b);
                        int ti = find_u64(n, s, t);
                        if (ti < 0) continue;
                        S2[c2].t = ti;
                        S2[c2].v = spin == 0 ? sc_element(M, h, g, t, 0, m, 0)
                                             : sc_element(M, h, g, 0, t, 0, m);
                        ++c2;
                    }
                }
            }
        }
        T->ns_of[x] = c1;
        T->nd_of[x] = c2;
    }
    return 0;
}

static void spin_free(sc_spin_t* T) {
    free(T->ns_of);
    free(T->nd_of);
    free(T->sing);
    free(T->dbl);
    free(T->coul);
}

/* Tables for sc_direct_sigma; diag [na*nb] (H_II including the constant) must
   stay valid while they are used.  NULL when memory runs out. */
void* sc_direct_setup(int M, const double* h, const double* g, int na, const uint64_t* amask,
                      int nb, const uint64_t* bmask, const double* diag) {
    sc_direct_t* D = (sc_direct_t*)calloc(1, sizeof(sc_direct_t));
    if (!D) return NULL;
    D->M = M;
    D->na = na;
    D->nb = nb;
    D->diag = diag;
    if (spin_setup(&D->A, M, h, g, na, amask, 0) || spin_setup(&D->B, M, h, g, nb, bmask, 1)) {
        spin_free(&D->A);
        spin_free(&D->B);
        free(D);
        return NULL;
    }
    return D;
}

void sc_direct_free(void* p) {
    sc_direct_t* D = (sc_direct_t*)p;
    if (!D) return;
    spin_free(&D->A);
    spin_free(&D->B);
    free(D);
}

/* out[I] = sum_J H_IJ c_J for the rows I of alpha strings [ia_lo, ia_hi). */
void sc_direct_sigma(const void* p, const double* c, double* out, int ia_lo, int ia_hi) {
    const sc_direct_t* D = (const sc_direct_t*)p;
    const int M = D->M, nb = D->nb;
    const double* g = D->A.g;
    for (int ia = ia_lo; ia < ia_hi; ++ia) {
        const sc_single_t* SA = D->A.sing + (size_t)ia * D->A.ns;
        const sc_double_t* DA = D->A.dbl + (size_t)ia * D->A.nd;
        const int nsa = D->A.ns_of[ia], nda = D->A.nd_of[ia];
        const double* ca_coul = D->A.coul + (size_t)ia * M * M;
        for (int ib = 0; ib < nb; ++ib) {
            const int64_t I = (int64_t)ia * nb + ib;
            const sc_single_t* SB = D->B.sing + (size_t)ib * D->B.ns;
            const sc_double_t* DB = D->B.dbl + (size_t)ib * D->B.nd;
            const int nsb = D->B.ns_of[ib], ndb = D->B.nd_of[ib];
            const double* cb_coul = D->B.coul + (size_t)ib * M * M;
            double acc = D->diag[I] * c[I];
            /* alpha singles: one-spin part plus the beta electrons' Coulomb term */
            for (int x = 0; x < nsa; ++x) {
                const sc_single_t* e = SA + x;
                acc += (e->v1 + e->sgn * cb_coul[e->a * M + e->i]) * c[(int64_t)e->t * nb + ib];
            }
            /* beta singles */
            for (int x = 0; x < nsb; ++x) {
                const sc_single_t* e = SB + x;
                acc += (e->v1 + e->sgn * ca_coul[e->a * M + e->i]) * c[(int64_t)ia * nb + e->t];
            }
            /* same-spin doubles */
            for (int x = 0; x < nda; ++x) acc += DA[x].v * c[(int64_t)DA[x].t * nb + ib];
            for (int x = 0; x < ndb; ++x) acc += DB[x].v * c[(int64_t)ia * nb + DB[x].t];
            /* opposite-spin doubles */
            for (int x = 0; x < nsa; ++x) {
                const sc_single_t* ea = SA + x;
                const double* crow = c + (int64_t)ea->t * nb;
                const double* gai = g + ((size_t)ea->a * M + ea->i) * M * M;
                double part = 0.0;
                for (int y = 0; y < nsb; ++y) {
                    const sc_single_t* eb = SB + y;
                    part += eb->sgn * gai[eb->a * M + eb->i] * crow[eb->t];
                }
                acc += ea->sgn * part;
            }
            out[I] = acc;
        }
    }
}
