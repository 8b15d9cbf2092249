/*
 * oracle.c -- plain CPU reference for the determinant-basis sigma vector
 * sigma = H C of direct configuration interaction (Vogiatzis et al.,
 * arXiv:1707.04346, Sec. 2.1, Eqs. 2, 4 and 5), in FP64.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU baseline
 * leg of the benchmark do.  It shares no code with the GPU path.
 *
 * What it computes, and how:
 *   * The determinant space (Sec. 2.1, Eq. 2; Sec. 3.1 for the GAS occupation
 *     types T): every pair (alpha string, beta string) with n_alpha and n_beta
 *     electrons in norb spatial orbitals whose cumulative (alpha+beta)
 *     occupation of GAS spaces 1..g lies within [min_cum[g], max_cum[g]] for
 *     every g.  One GAS space whose bounds equal n_alpha+n_beta is the CAS.
 *   * Spatial symmetry (the S of the TTSS blocks, Sec. 3.1, Eq. 9; the D2h
 *     spaces of Sec. 4-5), when orbital irreps are given: the irrep of a
 *     string is the product of the irreps of its occupied orbitals (D2h and
 *     its subgroups: irreps 0..7, product = bitwise XOR), and the space keeps
 *     only determinants whose alpha and beta irreps multiply to the target
 *     irrep.  A string's type is then its per-space counts followed by its
 *     irrep.
 *   * Determinant order (an interface contract, the paper fixes none):
 *     occupation types sorted lexicographically by their per-space electron
 *     counts (then by irrep); blocks (alpha type, beta type) in
 *     alpha-type-major order; inside a block, row-major [I_alpha][I_beta];
 *     strings of one type in ascending bitmask order.
 *   * sigma_I = sum_J <I|H|J> C_J, over every J of the space that differs from
 *     I by at most two spin orbitals (Eq. 4 / Eq. 5; determinants that differ
 *     by more do not couple, Sec. 3.1).  <I|H|J> is the Slater-Condon matrix
 *     element of the spin-free Hamiltonian of Eq. 6 with the excitation
 *     operators of Eq. 7, real orbitals, chemists' notation (ij|kl).
 *     No blocking, no splitting into sigma_1/2/3, no reuse between elements.
 *
 *   * One- and two-particle density matrices of a vector (the densities that
 *     Sec. 2.2 and Sec. 3.4 feed to the orbital step): the definitions
 *       gamma_pq   = sum_s <C|a+_ps a_qs|C> / <C|C>,
 *       Gamma_pqrs = sum_st <C|a+_ps a+_rt a_st a_qs|C> / <C|C>,
 *     applied operator by operator to every determinant (below).
 *
 * Sign convention: a determinant is alpha-hat(I_alpha) beta-hat(I_beta)|vac>
 * where each string operator is the product of creation operators in
 * ascending orbital order (Eq. 2).  The sign of a^+_p a_q acting on a string
 * holding q is (-1)^(number of occupied orbitals strictly between p and q);
 * excitation pairs never pick up a sign from the other spin's string.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXG 32

typedef struct {
    int norb, nel[2];
    int ngas, gas_norb[OR_MAXG], gas_first[OR_MAXG], min_cum[OR_MAXG], max_cum[OR_MAXG];
    int sym, orbsym[32], target;  /* orbital irreps (0..7) and target irrep when sym != 0 */
    /* per spin: kept strings, sorted by bitmask */
    int nstr[2];
    uint32_t *str[2];
    int *stype[2];
    int *srank[2];
    int ntype[2];
    int *tocc[2];     /* ntype x (ngas + 1): per-space counts, then the irrep (0 without symmetry) */
    int *tcount[2];
    int *tstart[2];   /* start of each type inside tlist */
    uint32_t *tlist[2]; /* strings grouped by type, ascending bitmask inside a type */
    int64_t *boff;    /* ntype[0] x ntype[1]; -1 when the block is not in the space */
    int64_t ndet;
    int nblk;
    int *blk_a, *blk_b;
    int64_t *blk_off;
    double *h;        /* norb x norb */
    double *g;        /* norb^4, g[((p*n+q)*n+r)*n+s] = (pq|rs) */
} or_space;

static inline int popc(uint32_t x) { return __builtin_popcount(x); }

/* type of a string: occupation of each GAS space, then its irrep */
static void occ_tuple(const or_space *S, uint32_t s, int *out) {
    for (int g = 0; g < S->ngas; ++g) {
        uint32_t m = 0;
        for (int k = 0; k < S->gas_norb[g]; ++k) m |= 1u << (S->gas_first[g] + k);
        out[g] = popc(s & m);
    }
    int irrep = 0;
    if (S->sym)
        for (int p = 0; p < S->norb; ++p)
            if ((s >> p) & 1u) irrep ^= S->orbsym[p];
    out[S->ngas] = irrep;
}

/* Do an alpha type and a beta type form an allowed pair (GAS bounds, and the
 * product of their irreps is the target)? */
static int pair_allowed(const or_space *S, const int *ta, const int *tb) {
    int cum = 0;
    for (int g = 0; g < S->ngas; ++g) {
        cum += ta[g] + tb[g];
        if (cum < S->min_cum[g] || cum > S->max_cum[g]) return 0;
    }
    if (S->sym && (ta[S->ngas] ^ tb[S->ngas]) != S->target) return 0;
    return 1;
}

static int tuple_cmp(const int *a, const int *b, int n) {
    for (int i = 0; i < n; ++i) {
        if (a[i] < b[i]) return -1;
        if (a[i] > b[i]) return 1;
    }
    return 0;
}

/* next bit pattern with the same popcount (Gosper) */
static uint64_t next_comb(uint64_t x) {
    uint64_t u = x & (~x + 1);
    uint64_t v = x + u;
    return v + (((v ^ x) / u) >> 2);
}

void or_free(or_space *S);

/* Build the determinant space (orbsym NULL: no spatial symmetry).  Returns
 * NULL on bad arguments. */
or_space *or_create_sym(int norb, int na, int nb, int ngas, const int *gas_norb, const int *min_cum,
                        const int *max_cum, const int *orbsym, int target, const double *h, const double *g) {
    if (norb < 1 || norb > 32 || na < 0 || nb < 0 || na > norb || nb > norb) return NULL;
    if (ngas < 1 || ngas > OR_MAXG) return NULL;
    if (orbsym) {
        if (target < 0 || target > 7) return NULL;
        for (int p = 0; p < norb; ++p)
            if (orbsym[p] < 0 || orbsym[p] > 7) return NULL;
    }
    or_space *S = (or_space *)calloc(1, sizeof(or_space));
    S->norb = norb; S->nel[0] = na; S->nel[1] = nb; S->ngas = ngas;
    S->sym = orbsym != NULL;
    S->target = orbsym ? target : 0;
    for (int p = 0; p < norb; ++p) S->orbsym[p] = orbsym ? orbsym[p] : 0;
    int tot = 0;
    for (int gi = 0; gi < ngas; ++gi) {
        S->gas_first[gi] = tot;
        S->gas_norb[gi] = gas_norb[gi];
        S->min_cum[gi] = min_cum[gi];
        S->max_cum[gi] = max_cum[gi];
        tot += gas_norb[gi];
    }
    if (tot != norb) { free(S); return NULL; }
    int G = ngas + 1;   /* type width: per-space counts and the irrep */
    /* enumerate all strings of each spin and their occupation tuples */
    uint32_t *all[2]; int nall[2]; int *allocc[2];
    for (int s = 0; s < 2; ++s) {
        int ne = S->nel[s];
        /* count C(norb, ne) */
        double c = 1; for (int k = 0; k < ne; ++k) c = c * (norb - k) / (k + 1);
        int64_t cnt = (int64_t)llround(c);
        if (cnt > 50000000) { for (int t = 0; t < s; ++t) { free(all[t]); free(allocc[t]); } free(S); return NULL; }
        all[s] = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cnt);
        allocc[s] = (int *)malloc(sizeof(int) * (size_t)cnt * G);
        int64_t k = 0;
        if (ne == 0) { all[s][0] = 0; k = 1; }
        else {
            uint64_t x = (ne == 32) ? 0xffffffffull : ((1ull << ne) - 1ull);
            uint64_t lim = 1ull << norb;
            while (x < lim) { all[s][k++] = (uint32_t)x; if (ne == 0) break; x = next_comb(x); }
        }
        nall[s] = (int)k;
        for (int64_t i = 0; i < k; ++i) occ_tuple(S, all[s][i], allocc[s] + i * G);
    }
    /* distinct tuples per spin */
    int *tup[2]; int ntup[2];
    for (int s = 0; s < 2; ++s) {
        tup[s] = (int *)malloc(sizeof(int) * (size_t)nall[s] * G);
        ntup[s] = 0;
        for (int i = 0; i < nall[s]; ++i) {
            int found = 0;
            for (int t = 0; t < ntup[s]; ++t)
                if (!tuple_cmp(tup[s] + t * G, allocc[s] + i * G, G)) { found = 1; break; }
            if (!found) { memcpy(tup[s] + ntup[s] * G, allocc[s] + i * G, sizeof(int) * G); ntup[s]++; }
        }
        /* sort lexicographically (insertion sort; few types) */
        for (int i = 1; i < ntup[s]; ++i) {
            int tmp[OR_MAXG + 1]; memcpy(tmp, tup[s] + i * G, sizeof(int) * G);
            int j = i - 1;
            while (j >= 0 && tuple_cmp(tup[s] + j * G, tmp, G) > 0) {
                memcpy(tup[s] + (j + 1) * G, tup[s] + j * G, sizeof(int) * G); --j;
            }
            memcpy(tup[s] + (j + 1) * G, tmp, sizeof(int) * G);
        }
    }
    /* keep types that have at least one allowed partner */
    int *keep[2];
    for (int s = 0; s < 2; ++s) keep[s] = (int *)calloc(ntup[s] > 0 ? ntup[s] : 1, sizeof(int));
    for (int a = 0; a < ntup[0]; ++a)
        for (int b = 0; b < ntup[1]; ++b)
            if (pair_allowed(S, tup[0] + a * G, tup[1] + b * G)) { keep[0][a] = 1; keep[1][b] = 1; }
    for (int s = 0; s < 2; ++s) {
        int nt = 0;
        for (int t = 0; t < ntup[s]; ++t) nt += keep[s][t];
        S->ntype[s] = nt;
        S->tocc[s] = (int *)malloc(sizeof(int) * (size_t)(nt > 0 ? nt : 1) * G);
        S->tcount[s] = (int *)calloc(nt > 0 ? nt : 1, sizeof(int));
        S->tstart[s] = (int *)calloc(nt + 1, sizeof(int));
        int j = 0;
        for (int t = 0; t < ntup[s]; ++t)
            if (keep[s][t]) { memcpy(S->tocc[s] + j * G, tup[s] + t * G, sizeof(int) * G); ++j; }
        /* kept strings, ascending bitmask (all[] already is) */
        int nk = 0;
        int *tid = (int *)malloc(sizeof(int) * (size_t)nall[s]);
        for (int i = 0; i < nall[s]; ++i) {
            tid[i] = -1;
            for (int t = 0; t < nt; ++t)
                if (!tuple_cmp(S->tocc[s] + t * G, allocc[s] + i * G, G)) { tid[i] = t; break; }
            if (tid[i] >= 0) ++nk;
        }
        S->nstr[s] = nk;
        S->str[s] = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nk > 0 ? nk : 1));
        S->stype[s] = (int *)malloc(sizeof(int) * (size_t)(nk > 0 ? nk : 1));
        S->srank[s] = (int *)malloc(sizeof(int) * (size_t)(nk > 0 ? nk : 1));
        S->tlist[s] = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nk > 0 ? nk : 1));
        int k = 0;
        for (int i = 0; i < nall[s]; ++i) {
            if (tid[i] < 0) continue;
            S->str[s][k] = all[s][i];
            S->stype[s][k] = tid[i];
            S->srank[s][k] = S->tcount[s][tid[i]]++;
            ++k;
        }
        for (int t = 0; t < nt; ++t) S->tstart[s][t + 1] = S->tstart[s][t] + S->tcount[s][t];
        for (int i = 0; i < nk; ++i)
            S->tlist[s][S->tstart[s][S->stype[s][i]] + S->srank[s][i]] = S->str[s][i];
        free(tid);
    }
    /* blocks */
    int na_t = S->ntype[0], nb_t = S->ntype[1];
    S->boff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(na_t * nb_t > 0 ? na_t * nb_t : 1));
    S->blk_a = (int *)malloc(sizeof(int) * (size_t)(na_t * nb_t > 0 ? na_t * nb_t : 1));
    S->blk_b = (int *)malloc(sizeof(int) * (size_t)(na_t * nb_t > 0 ? na_t * nb_t : 1));
    S->blk_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(na_t * nb_t + 1));
    int64_t off = 0; int nblk = 0;
    for (int a = 0; a < na_t; ++a)
        for (int b = 0; b < nb_t; ++b) {
            if (pair_allowed(S, S->tocc[0] + a * G, S->tocc[1] + b * G)) {
                S->boff[a * nb_t + b] = off;
                S->blk_a[nblk] = a; S->blk_b[nblk] = b; S->blk_off[nblk] = off; ++nblk;
                off += (int64_t)S->tcount[0][a] * S->tcount[1][b];
            } else S->boff[a * nb_t + b] = -1;
        }
    S->blk_off[nblk] = off;
    S->nblk = nblk;
    S->ndet = off;
    /* integrals */
    size_t n2 = (size_t)norb * norb;
    S->h = (double *)malloc(sizeof(double) * n2);
    S->g = (double *)malloc(sizeof(double) * n2 * n2);
    memcpy(S->h, h, sizeof(double) * n2);
    memcpy(S->g, g, sizeof(double) * n2 * n2);
    for (int s = 0; s < 2; ++s) { free(all[s]); free(allocc[s]); free(tup[s]); free(keep[s]); }
    return S;
}

or_space *or_create(int norb, int na, int nb, int ngas, const int *gas_norb,
                    const int *min_cum, const int *max_cum, const double *h, const double *g) {
    return or_create_sym(norb, na, nb, ngas, gas_norb, min_cum, max_cum, NULL, 0, h, g);
}

void or_free(or_space *S) {
    if (!S) return;
    for (int s = 0; s < 2; ++s) {
        free(S->str[s]); free(S->stype[s]); free(S->srank[s]); free(S->tocc[s]);
        free(S->tcount[s]); free(S->tstart[s]); free(S->tlist[s]);
    }
    free(S->boff); free(S->blk_a); free(S->blk_b); free(S->blk_off);
    free(S->h); free(S->g); free(S);
}

int64_t or_ndet(const or_space *S) { return S->ndet; }
int or_nstr(const or_space *S, int spin) { return S->nstr[spin]; }
int or_ntype(const or_space *S, int spin) { return S->ntype[spin]; }
int or_nblocks(const or_space *S) { return S->nblk; }

/* block table: alpha type, beta type, offset (nblk+1 offsets) */
void or_blocks(const or_space *S, int *ta, int *tb, int64_t *offs) {
    for (int i = 0; i < S->nblk; ++i) { ta[i] = S->blk_a[i]; tb[i] = S->blk_b[i]; offs[i] = S->blk_off[i]; }
    offs[S->nblk] = S->blk_off[S->nblk];
}

/* strings of one spin, grouped by type (ascending bitmask inside a type) and per-type counts */
void or_strings(const or_space *S, int spin, uint32_t *out, int *tcount) {
    memcpy(out, S->tlist[spin], sizeof(uint32_t) * (size_t)S->nstr[spin]);
    memcpy(tcount, S->tcount[spin], sizeof(int) * (size_t)S->ntype[spin]);
}

/* index of a string in the kept sorted list, or -1 */
static int find_str(const or_space *S, int s, uint32_t x) {
    int lo = 0, hi = S->nstr[s] - 1;
    const uint32_t *a = S->str[s];
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] == x) return mid;
        if (a[mid] < x) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* position of determinant (alpha bits, beta bits) in the vector, or -1 */
int64_t or_address(const or_space *S, uint32_t ia, uint32_t ib) {
    int a = find_str(S, 0, ia), b = find_str(S, 1, ib);
    if (a < 0 || b < 0) return -1;
    int ta = S->stype[0][a], tb = S->stype[1][b];
    int64_t off = S->boff[ta * S->ntype[1] + tb];
    if (off < 0) return -1;
    return off + (int64_t)S->srank[0][a] * S->tcount[1][tb] + S->srank[1][b];
}

/* alpha and beta bit patterns of determinant idx */
static void det_of(const or_space *S, int64_t idx, uint32_t *ia, uint32_t *ib) {
    int lo = 0, hi = S->nblk - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (S->blk_off[mid] <= idx) lo = mid; else hi = mid - 1;
    }
    int ta = S->blk_a[lo], tb = S->blk_b[lo];
    int64_t rel = idx - S->blk_off[lo];
    int64_t nbs = S->tcount[1][tb];
    *ia = S->tlist[0][S->tstart[0][ta] + (int)(rel / nbs)];
    *ib = S->tlist[1][S->tstart[1][tb] + (int)(rel % nbs)];
}

void or_det(const or_space *S, int64_t idx, uint32_t *ia, uint32_t *ib) { det_of(S, idx, ia, ib); }

/* ---------------------------------------------------------------------------
 * Slater-Condon matrix elements of Eq. 6 between determinants.
 * ------------------------------------------------------------------------- */

#define G4(S, p, q, r, s) ((S)->g[(((size_t)(p) * (S)->norb + (q)) * (S)->norb + (r)) * (S)->norb + (s)])
#define H2(S, p, q) ((S)->h[(size_t)(p) * (S)->norb + (q)])

/* sign of a^+_p a_q acting on string x (q occupied): parity of the occupied
 * orbitals strictly between p and q */
static double exc_sign(uint32_t x, int p, int q) {
    int lo = p < q ? p : q, hi = p < q ? q : p;
    if (hi - lo <= 1) return 1.0;
    uint32_t below_hi = (hi >= 32) ? 0xffffffffu : ((1u << hi) - 1u);
    uint32_t upto_lo = (lo + 1 >= 32) ? 0xffffffffu : ((1u << (lo + 1)) - 1u);
    return (popc(x & below_hi & ~upto_lo) & 1) ? -1.0 : 1.0;
}

static int lowbit(uint32_t x) { return __builtin_ctz(x); }
static int highbit(uint32_t x) { return 31 - __builtin_clz(x); }

/* <I|H|J> for I = (ia, ib), J = (ja, jb) */
static double h_elem(const or_space *S, uint32_t ia, uint32_t ib, uint32_t ja, uint32_t jb) {
    uint32_t da = ia ^ ja, db = ib ^ jb;
    int nda = popc(da) / 2, ndb = popc(db) / 2;
    if (nda + ndb > 2) return 0.0;
    int n = S->norb;
    if (nda == 0 && ndb == 0) {
        /* diagonal: one-electron energies, same-spin Coulomb minus exchange,
         * opposite-spin Coulomb */
        double e = 0.0;
        for (int p = 0; p < n; ++p) {
            int pa = (ia >> p) & 1, pb = (ib >> p) & 1;
            if (pa) e += H2(S, p, p);
            if (pb) e += H2(S, p, p);
            for (int q = 0; q < n; ++q) {
                int qa = (ia >> q) & 1, qb = (ib >> q) & 1;
                if (pa && qa) e += 0.5 * (G4(S, p, p, q, q) - G4(S, p, q, q, p));
                if (pb && qb) e += 0.5 * (G4(S, p, p, q, q) - G4(S, p, q, q, p));
                if (pa && qb) e += G4(S, p, p, q, q);
            }
        }
        return e;
    }
    if (ndb == 0 && nda == 1) {
        int p = lowbit(ia & ~ja), q = lowbit(ja & ~ia);   /* I = a^+_p a_q J */
        double v = H2(S, p, q);
        for (int r = 0; r < n; ++r) {
            if ((ja >> r) & 1) v += G4(S, p, q, r, r) - G4(S, p, r, r, q);
            if ((jb >> r) & 1) v += G4(S, p, q, r, r);
        }
        return exc_sign(ja, p, q) * v;
    }
    if (nda == 0 && ndb == 1) {
        int p = lowbit(ib & ~jb), q = lowbit(jb & ~ib);
        double v = H2(S, p, q);
        for (int r = 0; r < n; ++r) {
            if ((jb >> r) & 1) v += G4(S, p, q, r, r) - G4(S, p, r, r, q);
            if ((ja >> r) & 1) v += G4(S, p, q, r, r);
        }
        return exc_sign(jb, p, q) * v;
    }
    if (nda == 1 && ndb == 1) {
        int p = lowbit(ia & ~ja), q = lowbit(ja & ~ia);
        int r = lowbit(ib & ~jb), t = lowbit(jb & ~ib);
        return exc_sign(ja, p, q) * exc_sign(jb, r, t) * G4(S, p, q, r, t);
    }
    /* two differences in one spin string */
    uint32_t i_, j_;
    if (nda == 2) { i_ = ia; j_ = ja; } else { i_ = ib; j_ = jb; }
    uint32_t pi = i_ & ~j_, qj = j_ & ~i_;
    int p1 = lowbit(pi), p2 = highbit(pi), q1 = lowbit(qj), q2 = highbit(qj);
    double s1 = exc_sign(j_, p1, q1);
    uint32_t k_ = (j_ & ~(1u << q1)) | (1u << p1);
    double s2 = exc_sign(k_, p2, q2);
    return s1 * s2 * (G4(S, p1, q1, p2, q2) - G4(S, p1, q2, p2, q1));
}

double or_h_elem(const or_space *S, int64_t i, int64_t j) {
    uint32_t ia, ib, ja, jb;
    det_of(S, i, &ia, &ib);
    det_of(S, j, &ja, &jb);
    return h_elem(S, ia, ib, ja, jb);
}

/* sigma_I = sum_J <I|H|J> C_J for one output determinant I, summing over every
 * J of the space reachable from I by at most two electron moves. */
static double sigma_row(const or_space *S, uint32_t ia, uint32_t ib, const double *C) {
    int n = S->norb;
    uint32_t full = (n >= 32) ? 0xffffffffu : ((1u << n) - 1u);
    double acc = 0.0;
    int64_t j;
    /* J = I */
    j = or_address(S, ia, ib);
    if (j >= 0) acc += h_elem(S, ia, ib, ia, ib) * C[j];
    uint32_t occ[2] = {ia, ib}, vir[2] = {full & ~ia, full & ~ib};
    /* one spin string changes by one or two electrons */
    for (int s = 0; s < 2; ++s) {
        for (uint32_t o1 = occ[s]; o1; o1 &= o1 - 1) {
            int p = lowbit(o1);
            for (uint32_t v1 = vir[s]; v1; v1 &= v1 - 1) {
                int q = lowbit(v1);
                uint32_t x = (occ[s] & ~(1u << p)) | (1u << q);
                uint32_t ja = s == 0 ? x : ia, jb = s == 0 ? ib : x;
                j = or_address(S, ja, jb);
                if (j >= 0) acc += h_elem(S, ia, ib, ja, jb) * C[j];
                /* second move in the same string, counted once: p2 > p, q2 > q */
                for (uint32_t o2 = o1 & (o1 - 1); o2; o2 &= o2 - 1) {
                    int p2 = lowbit(o2);
                    for (uint32_t v2 = v1 & (v1 - 1); v2; v2 &= v2 - 1) {
                        int q2 = lowbit(v2);
                        uint32_t y = (x & ~(1u << p2)) | (1u << q2);
                        uint32_t ka = s == 0 ? y : ia, kb = s == 0 ? ib : y;
                        j = or_address(S, ka, kb);
                        if (j >= 0) acc += h_elem(S, ia, ib, ka, kb) * C[j];
                    }
                }
            }
        }
    }
    /* one alpha and one beta electron move */
    for (uint32_t o1 = ia; o1; o1 &= o1 - 1) {
        int p = lowbit(o1);
        for (uint32_t v1 = full & ~ia; v1; v1 &= v1 - 1) {
            int q = lowbit(v1);
            uint32_t ja = (ia & ~(1u << p)) | (1u << q);
            for (uint32_t o2 = ib; o2; o2 &= o2 - 1) {
                int r = lowbit(o2);
                for (uint32_t v2 = full & ~ib; v2; v2 &= v2 - 1) {
                    int t = lowbit(v2);
                    uint32_t jb = (ib & ~(1u << r)) | (1u << t);
                    j = or_address(S, ja, jb);
                    if (j >= 0) acc += h_elem(S, ia, ib, ja, jb) * C[j];
                }
            }
        }
    }
    return acc;
}

void or_set_threads(int nt) {
#ifdef _OPENMP
    if (nt > 0) omp_set_num_threads(nt);
#else
    (void)nt;
#endif
}

int or_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* full sigma vector */
void or_sigma(const or_space *S, const double *C, double *sigma) {
    int64_t N = S->ndet;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < N; ++i) {
        uint32_t ia, ib;
        det_of(S, i, &ia, &ib);
        sigma[i] = sigma_row(S, ia, ib, C);
    }
}

/* sigma at selected output determinants only */
void or_sigma_rows(const or_space *S, int64_t nrows, const int64_t *rows, const double *C, double *out) {
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nrows; ++k) {
        uint32_t ia, ib;
        det_of(S, rows[k], &ia, &ib);
        out[k] = sigma_row(S, ia, ib, C);
    }
}

/* diagonal H_II */
void or_hdiag(const or_space *S, double *out) {
    int64_t N = S->ndet;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        uint32_t ia, ib;
        det_of(S, i, &ia, &ib);
        out[i] = h_elem(S, ia, ib, ia, ib);
    }
}

/* dense H (row-major N x N) for tiny spaces */
int or_hmat(const or_space *S, double *out) {
    int64_t N = S->ndet;
    if (N > 20000) return -1;
    #pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < N; ++i) {
        uint32_t ia, ib;
        det_of(S, i, &ia, &ib);
        for (int64_t j = 0; j < N; ++j) {
            uint32_t ja, jb;
            det_of(S, j, &ja, &jb);
            out[i * N + j] = h_elem(S, ia, ib, ja, jb);
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Density matrices by direct operator application.
 *
 * A determinant is held as one 64-bit word of spin orbitals: alpha orbital p
 * is bit p, beta orbital p is bit norb + p, so that the ascending creation
 * order of Eq. 2 (alpha string left of beta string) is ascending bit order.
 * a_k and a+_k act with the sign (-1)^(occupied spin orbitals below k).
 * ------------------------------------------------------------------------- */

/* a_k on d: 0 when k is empty, else the new word and the sign */
static int op_ann(uint64_t d, int k, uint64_t *out, int *sign) {
    uint64_t b = (uint64_t)1 << k;
    if (!(d & b)) return 0;
    *sign *= (__builtin_popcountll(d & (b - 1)) & 1) ? -1 : 1;
    *out = d & ~b;
    return 1;
}

/* a+_k on d: 0 when k is occupied */
static int op_cre(uint64_t d, int k, uint64_t *out, int *sign) {
    uint64_t b = (uint64_t)1 << k;
    if (d & b) return 0;
    *sign *= (__builtin_popcountll(d & (b - 1)) & 1) ? -1 : 1;
    *out = d | b;
    return 1;
}

static int64_t index_of_word(const or_space *S, uint64_t d) {
    uint32_t ia = (uint32_t)(d & ((S->norb >= 32) ? 0xffffffffu : ((1u << S->norb) - 1u)));
    uint32_t ib = (uint32_t)(d >> S->norb);
    if (popc(ia) != S->nel[0] || popc(ib) != S->nel[1]) return -1;
    return or_address(S, ia, ib);
}

/* rdm1[n*n], rdm2[n^4] (index ((p*n+q)*n+r)*n+s), both normalised by <C|C>;
 * returns 0, or -1 for a zero vector */
int or_rdm(const or_space *S, const double *C, double *rdm1, double *rdm2) {
    const int n = S->norb, n2 = 2 * n;
    const int64_t N = S->ndet;
    const size_t n4 = (size_t)n * n * n * n;
    double cc = 0;
    for (int64_t j = 0; j < N; ++j) cc += C[j] * C[j];
    if (!(cc > 0)) return -1;
    memset(rdm1, 0, sizeof(double) * n * n);
    memset(rdm2, 0, sizeof(double) * n4);
    #pragma omp parallel
    {
        double *g1 = calloc((size_t)n * n, sizeof(double));
        double *g2 = calloc(n4, sizeof(double));
        #pragma omp for schedule(dynamic, 16)
        for (int64_t j = 0; j < N; ++j) {
            if (C[j] == 0) continue;
            uint32_t ja, jb;
            det_of(S, j, &ja, &jb);
            const uint64_t d0 = (uint64_t)ja | ((uint64_t)jb << n);
            /* one-body: a+_P a_Q with P, Q spin orbitals of one spin */
            for (int Q = 0; Q < n2; ++Q) {
                uint64_t d1; int s1 = 1;
                if (!op_ann(d0, Q, &d1, &s1)) continue;
                const int sp = Q / n, q = Q % n;
                for (int p = 0; p < n; ++p) {
                    uint64_t d2; int s2 = s1;
                    if (!op_cre(d1, sp * n + p, &d2, &s2)) continue;
                    int64_t i = index_of_word(S, d2);
                    if (i >= 0) g1[(size_t)p * n + q] += C[i] * s2 * C[j];
                }
            }
            /* two-body: a+_P a+_R a_T a_Q, P and Q of spin s, R and T of spin t */
            for (int Q = 0; Q < n2; ++Q) {
                uint64_t d1; int s1 = 1;
                if (!op_ann(d0, Q, &d1, &s1)) continue;
                const int sq = Q / n, q = Q % n;
                for (int T = 0; T < n2; ++T) {
                    uint64_t d2; int s2 = s1;
                    if (!op_ann(d1, T, &d2, &s2)) continue;
                    const int st = T / n, t = T % n;
                    for (int r = 0; r < n; ++r) {
                        uint64_t d3; int s3 = s2;
                        if (!op_cre(d2, st * n + r, &d3, &s3)) continue;
                        for (int p = 0; p < n; ++p) {
                            uint64_t d4; int s4 = s3;
                            if (!op_cre(d3, sq * n + p, &d4, &s4)) continue;
                            int64_t i = index_of_word(S, d4);
                            if (i >= 0) g2[(((size_t)p * n + q) * n + r) * n + t] += C[i] * s4 * C[j];
                        }
                    }
                }
            }
        }
        #pragma omp critical
        {
            for (size_t k = 0; k < (size_t)n * n; ++k) rdm1[k] += g1[k];
            for (size_t k = 0; k < n4; ++k) rdm2[k] += g2[k];
        }
        free(g1);
        free(g2);
    }
    for (size_t k = 0; k < (size_t)n * n; ++k) rdm1[k] /= cc;
    for (size_t k = 0; k < n4; ++k) rdm2[k] /= cc;
    return 0;
}
