/*
 * cisigma.h -- C ABI of the MI355X determinant-CI sigma builder and Davidson
 * eigensolver.
 *
 * The library computes the direct-CI sigma vector sigma = H C of Vogiatzis et
 * al., arXiv:1707.04346 (Sec. 2.1, Eqs. 4-8), over alpha/beta occupation
 * strings (Eq. 2) of a CAS or GAS space (Sec. 3.1), and the lowest
 * eigenpairs of H by the Davidson method the sigma vector serves (Sec. 2.1 and
 * Sec. 3.3).  All numerical work runs in HIP kernels on one GPU; host memory
 * is touched only to take in the integrals and to hand back energies.
 *
 * Hamiltonian (Eq. 6, with the spin-summed excitation operators of Eq. 7):
 *     H = sum_kl h_kl E_kl + 1/2 sum_ijkl (ij|kl) (E_ij E_kl - delta_jk E_il)
 * real orbitals, chemists' notation (ij|kl).
 *
 * Determinant space and order (a contract of this library; the paper fixes no
 * order):
 *   - norb spatial orbitals numbered 0..norb-1; GAS space g holds the next
 *     gas->norb[g] orbitals after space g-1.
 *   - a string is a bitmask of occupied orbitals (bit p = orbital p); its
 *     occupation type is the tuple of electron counts per GAS space (Sec. 3.1,
 *     Eq. 9: the T of a TS string).
 *   - the space holds every (alpha string, beta string) with nalpha and nbeta
 *     electrons such that, for every g, the total (alpha + beta) count in
 *     spaces 0..g lies in [gas->min_cum[g], gas->max_cum[g]].
 *   - occupation types of one spin are ordered lexicographically by their
 *     tuples; only types that pair with at least one type of the other spin
 *     are kept.  Strings of a type are ordered by ascending bitmask.  The
 *     string index of a spin runs over types in that order.
 *   - the vector is a sequence of blocks (alpha type, beta type) -- the TTSS
 *     blocks of Sec. 3.1 without the spatial-symmetry label -- in
 *     alpha-type-major order, each block row-major [I_alpha][I_beta].  A CAS
 *     is one block of N_alpha x N_beta elements.
 *   - determinant |alpha(I_a) beta(I_b)> = a^+_{p1 a} ... a^+_{pk a} a^+_{q1 b}
 *     ... |vac> with p1 < p2 < ..., alpha operators to the left (Eq. 2).
 *
 * Memory and streams: every vector argument named "device" is a pointer to
 * GPU memory owned by the caller (for example a torch tensor's data_ptr()).
 * Streams are hipStream_t passed as void*; NULL means the default (null)
 * stream.  Host arrays are read during the call and may be freed afterwards.
 *
 * Errors: every call returns CISIGMA_OK (0) or a negative status; no C++
 * exception crosses this boundary.  cisigma_last_error() returns a message
 * for the most recent failure on a context.  A context is not thread-safe;
 * use one per host thread.
 */
#ifndef CISIGMA_H
#define CISIGMA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define CISIGMA_OK 0
#define CISIGMA_EINVAL (-1)   /* bad argument: sizes, NULL, NaN, asymmetric integrals, aliasing, empty space */
#define CISIGMA_ENOMEM (-2)   /* device (or host) allocation failed */
#define CISIGMA_EDEVICE (-3)  /* a HIP call failed; the message is kept */
#define CISIGMA_ENOCONV (-4)  /* Davidson reached max_iter; energies are still written */
#define CISIGMA_EUNSUPPORTED (-5) /* valid request outside what this build implements */

/* element types of CI vectors */
#define CISIGMA_FP64 0
#define CISIGMA_FP32 1

/* option keys for cisigma_set_option */
#define CISIGMA_OPT_PRECISION 1    /* Davidson vectors and sigma: CISIGMA_FP64 (plain) or CISIGMA_FP32 (mixed) */
#define CISIGMA_OPT_MAX_SPACE 2    /* Davidson subspace size before collapse (>= 2*nroots); default max(8*nroots, 32),
                                      capped by what fits in 70% of free device memory */
#define CISIGMA_OPT_MAX_ITER 3     /* Davidson iteration limit; default 100 */
#define CISIGMA_OPT_REFINE_EVERY 4 /* mixed mode: also refine in FP64 every R iterations; default 0 = only when the
                                      FP32 iteration meets the convergence test */
#define CISIGMA_OPT_RESID_TOL 5    /* residual-norm threshold; default sqrt(tol) (mixed: max(sqrt(tol), 1e-5)) */
#define CISIGMA_OPT_VERBOSE 6      /* print one line per Davidson iteration to stderr when nonzero */
#define CISIGMA_OPT_PROFILE 7      /* nonzero: time every pass of cisigma_apply with HIP events (resets the totals) */
#define CISIGMA_OPT_SIGMA_PATH 8   /* 0: automatic kernel choice; 1: only the general (scatter-atomic) kernels;
                                      2: for one-block spaces, the owner-computes units of the GAS form
                                      in place of the one-block owner kernel (rebuilds the unit tables);
                                      3: as 0, but the one-block owner kernel in FP32 in its two-W-tile
                                      form (one workgroup per compute unit) even where two workgroups of
                                      the one-W-tile form would fit */
#define CISIGMA_OPT_UNIT_LAUNCH 19 /* owner-computes units: 0 (default) one launch over every unit, longest
                                      rows of work first; 1: one launch per unit, in the same order (the
                                      per-block launch baseline) */
#define CISIGMA_OPT_DETERMINISTIC 20 /* 1: cisigma_apply (and the Davidson's sigma builds) use only kernels
                                      without floating-point atomics, whose results repeat bit for bit;
                                      an apply that would need a float-atomic kernel (shapes outside the
                                      owner-computes and stored-row kernels, stored rows that do not fit
                                      in memory, CISIGMA_OPT_SIGMA_PATH = 1) fails with
                                      CISIGMA_EUNSUPPORTED instead; the sigma output is then not written.
                                      0 (default): such applies run the atomic kernels */
#define CISIGMA_OPT_UNIT_COLS 18   /* owner-computes units (GAS spaces, one-block spaces whose sigma row is
                                      longer than the LDS, or path 2): at most this many sigma columns per
                                      unit, 64..65536; 0 (default): as many as the LDS holds.  Rows are cut
                                      at beta-type ends (GAS) or at the occupation classes of the two
                                      highest orbitals (one-block), and inside a piece only when it alone
                                      is longer.  Rebuilds the unit tables; set by cisigma_autotune */
#define CISIGMA_OPT_SS_CHUNK 9     /* materialised same-spin products of one-block spaces: at most this many
                                      columns per chunk (a positive multiple of 64), within the chunk the
                                      workspace was sized for; 0 (default): the workspace's chunk, whose
                                      slab of the gathered copy stays near 192 MiB (the Infinity Cache)
                                      when that copy is below 2 GB, and what fits in memory */
#define CISIGMA_OPT_OVERLAP 12     /* nonzero: cisigma_apply runs the beta-beta pass on a second
                                      stream of the context, overlapping the alpha-beta pass, and joins
                                      before the output gather (the call stays ordered on `stream`);
                                      0 (default): one stream.  Measured gain ~1.5% at CAS(16,16), while
                                      the alpha-beta kernel runs ~25% longer beside it.  With profiling on,
                                      the beta-beta entry of
                                      cisigma_pass_times is then the wait for that stream after the
                                      alpha-beta pass */
#define CISIGMA_OPT_GAS_UNIT_ORDER 16 /* launch order of the GAS owner-computes units (both precisions):
                                      0 (default) most source tiles per row first, 1 alpha-type order,
                                      2 most total work first, 3 heavy and light alternating, 4 heaviest
                                      first by the batch weight sum_j c_j l_j of Sec. 3.1 Eq. 10, 5 by
                                      (sum_j c_j) N_blocks of Eq. 11 (a unit as the batch, its blocks'
                                      connections c_j and determinants l_j); set by cisigma_autotune per
                                      precision */
#define CISIGMA_OPT_SS_SPLIT 17     /* column split of the grid of the same-spin pair-product kernel of
                                      spaces with several types (GAS or point-group symmetry; row-store
                                      or atomic form), 1..64; 0 (default): a heuristic; set by
                                      cisigma_autotune */
#define CISIGMA_OPT_LOW_MEMORY 15   /* nonzero: the mixed-precision Davidson frees the FP32 sigma workspace
                                      before each FP64 refinement and the FP64 one after it, so only one is
                                      held at a time; done anyway when the FP64 workspace does not fit in
                                      free memory (CAS(18,18) with a 6-vector subspace).  Default 0 */
#define CISIGMA_OPT_PSPACE 14       /* Davidson P-space (Sec. 2.1 step (2), preconditioner): the exact block
                                      of H over the P determinants with the lowest H_II (P <= 2048; default
                                      256; 0: none) gives the initial guess (its lowest eigenvectors) and,
                                      on those determinants, the correction (theta - H_PP)^-1 r_P in place
                                      of the diagonal one.  Not used with CISIGMA_OPT_SPIN_PARITY != 0.
                                      Measured: 3 roots at CAS(16,16) take 347 instead of 360 sigma builds
                                      (mixed precision 24.7 instead of 25.3 s) */
#define CISIGMA_OPT_THICK_RESTART 13 /* nonzero (default): when the Davidson basis would exceed max_space it
                                      collapses onto the current Ritz vectors plus the part of the previous
                                      iteration's Ritz vectors outside them (at most 2 nroots vectors; used
                                      when nroots <= 8 and 3 nroots <= max_space); 0: the current Ritz
                                      vectors only */
#define CISIGMA_OPT_GRAPH 11       /* nonzero: cisigma_apply on a non-NULL stream runs its kernels eagerly
                                      at the first call with a given (C, sigma, dtype, stream) and captures
                                      them into a HIP graph that later calls with the same arguments replay
                                      (for callers applying sigma to the same buffers many times, where
                                      launch overhead matters: small spaces).  NULL stream, profiling on:
                                      eager.  Changing the spin-parity, sigma-path or chunk options drops
                                      the captured graphs.  Default 0 */
#define CISIGMA_OPT_SPIN_PARITY 10 /* M_S = 0 spin symmetry (Sec. 3.1, Sec. 3.3): p = +1 or -1 restricts
                                      cisigma_apply and cisigma_davidson to vectors with
                                      C(Ib, Ia) = p C(Ia, Ib) (p = +1: even total spin S, singlets first;
                                      p = -1: odd S), which drops the beta-beta pass; 0 (default): none.
                                      H conserves S^2 and the Davidson guess is built on the lowest
                                      diagonal elements, so a sector run can miss a root of a spin its
                                      guess lacks (a quintet below the lowest singlet): ask for more
                                      roots to include such states.
                                      Needs nalpha = nbeta (EINVAL otherwise).  GAS and point-group
                                      spaces qualify (their blocks (ta, tb) and (tb, ta) mirror each
                                      other): C(Ib, Ia) is then the element of block (tb, ta); a space
                                      whose alpha and beta tables do not mirror each other gives
                                      EUNSUPPORTED */

/* passes of one cisigma_apply, in order, as reported by cisigma_pass_times */
#define CISIGMA_PASS_LAYOUT_IN 0   /* C -> padded alpha-major and beta-major copies */
#define CISIGMA_PASS_CLEAR 1       /* clear the two accumulators */
#define CISIGMA_PASS_SIGMA_AA 2    /* sigma_2: alpha-alpha part (Eq. 8) */
#define CISIGMA_PASS_SIGMA_AB 3    /* sigma_3: alpha-beta part */
#define CISIGMA_PASS_SIGMA_BB 4    /* sigma_1: beta-beta part */
#define CISIGMA_PASS_LAYOUT_OUT 5  /* accumulators -> sigma */
#define CISIGMA_NPASS 6

/* GAS definition (Sec. 3.1).  Cumulative bounds are on total (alpha+beta)
 * electrons.  Pass NULL to cisigma_init for a CAS. */
typedef struct cisigma_gas {
    int ngas;             /* 1..16 */
    const int *norb;      /* [ngas] orbitals per space, summing to norb */
    const int *min_cum;   /* [ngas] */
    const int *max_cum;   /* [ngas] */
} cisigma_gas;

typedef struct cisigma_stats {
    int iterations;       /* Davidson iterations performed */
    int sigma_fp32;       /* sigma builds in FP32 */
    int sigma_fp64;       /* sigma builds in FP64 */
    int refinements;      /* FP64 refinement points (mixed mode) */
    double residual;      /* final max residual norm (from an FP64 sigma) */
    double seconds;       /* wall time of the call */
} cisigma_stats;

typedef struct cisigma_ctx cisigma_ctx;

/*
 * cisigma_init -- build a context for (norb, nalpha, nbeta, GAS) and integrals.
 *   ctx    out: new context (NULL on failure).
 *   norb   1..32 orbitals; 0 <= nalpha, nbeta <= norb.
 *   gas    NULL for a CAS (one space holding all electrons), else Sec. 3.1 GAS.
 *   h1e    host FP64 [norb*norb], row-major, symmetric (|h_pq - h_qp| <= 1e-12 max|h|).
 *   eri    host FP64 [norb^4], eri[((i*n+j)*n+k)*n+l] = (ij|kl), 8-fold symmetric.
 * Both integral arrays are copied; the caller keeps ownership.  Builds the
 * string, excitation-list and integral tables on the current HIP device
 * (synchronous).  Returns EINVAL for bad sizes, NaN or asymmetric integrals
 * or an empty space; ENOMEM when device memory runs out; EDEVICE on a HIP
 * failure.
 */
int cisigma_init(cisigma_ctx **ctx, int norb, int nalpha, int nbeta, const cisigma_gas *gas,
                 const double *h1e, const double *eri);

/*
 * cisigma_init_sym -- cisigma_init with spatial (point-group) symmetry, the S of
 * the TTSS blocks of Sec. 3.1 (Eq. 9) for the D2h spaces of Sec. 4-5.
 *   orbsym  host int[norb]: the irrep of each orbital, 0..7, in a labelling
 *           where the product of two irreps is their bitwise XOR (D2h and its
 *           subgroups C2v, C2h, D2, Cs, Ci, C2, C1), 0 the totally symmetric
 *           irrep.  NULL: no symmetry (exactly cisigma_init).
 *   target  the irrep of the space, 0..7.
 * The irrep of a string is the product of the irreps of its occupied orbitals.
 * The space keeps the determinants of cisigma_init whose alpha and beta string
 * irreps multiply to target.  A string type is then (GAS occupation tuple,
 * irrep): types are ordered by tuple, then by irrep, strings of a type by
 * ascending bitmask, and blocks (alpha type, beta type) as in cisigma_init
 * (alpha-type-major, row-major inside).  The integrals must respect the
 * symmetry: h_pq = 0 unless orbsym[p] == orbsym[q] and (pq|rs) = 0 unless
 * orbsym[p]^orbsym[q]^orbsym[r]^orbsym[s] == 0, to 1e-12 of the largest
 * element (EINVAL otherwise), so that H does not couple the space to the
 * rest.  Sigma and Davidson then act on the symmetric space only.  EINVAL
 * also for irreps outside 0..7 or an empty space.
 */
int cisigma_init_sym(cisigma_ctx **ctx, int norb, int nalpha, int nbeta, const cisigma_gas *gas,
                     const int *orbsym, int target, const double *h1e, const double *eri);

/* release all device memory of the context; NULL is ignored */
void cisigma_free(cisigma_ctx *ctx);

/* number of determinants (vector length), or -1 for a NULL context */
int64_t cisigma_ndet(const cisigma_ctx *ctx);

/*
 * cisigma_layout -- the block table of the vector order above.
 *   nblocks    out: number of (alpha type, beta type) blocks.
 *   The array arguments may be NULL (then only nblocks is written); otherwise
 *   they need room for *nblocks (block_offset: *nblocks + 1) entries:
 *   block_offset[b] first element of block b (block_offset[nblocks] = ndet),
 *   alpha_type/beta_type type indices, nalpha_str/nbeta_str strings per type
 *   of the block's alpha and beta type.
 */
int cisigma_layout(const cisigma_ctx *ctx, int *nblocks, int64_t *block_offset, int *alpha_type,
                   int *beta_type, int *nalpha_str, int *nbeta_str);

/*
 * cisigma_address -- position of determinant (alpha bits, beta bits) in the
 * vector; *index = -1 when it is not in the space.  Host-side, no device work.
 */
int cisigma_address(const cisigma_ctx *ctx, uint32_t alpha_bits, uint32_t beta_bits, int64_t *index);

/*
 * cisigma_strings -- copy the device string table of one spin (0 alpha,
 * 1 beta) to the host: out[nstr] bitmasks in string-index order.  *nstr is
 * written; out may be NULL to query the size only.
 */
int cisigma_strings(const cisigma_ctx *ctx, int spin, uint32_t *out, int *nstr);

/*
 * cisigma_excitations -- copy the device single-excitation list of one spin
 * to the host (the E_kl connection lists of Sec. 3.1 / Sec. 3.3).  For string
 * I and each occupied k (ascending) and empty l (ascending), the entry at
 * [I][ko*nvirt + lv] describes J = I - k + l:
 *     bits 31..11  index of J (all ones = J is not a string of the space)
 *     bits 10..6   k,  bits 5..1  l,  bit 0  1 when <J|a^+_l a_k|I> = -1
 * (the whole word is 0xFFFFFFFF when J is not in the space).
 * out may be NULL; *per_string = nelec*(norb-nelec) and *nstr are written.
 */
int cisigma_excitations(const cisigma_ctx *ctx, int spin, uint32_t *out, int *per_string, int *nstr);

/* option setter; EINVAL for an unknown key or out-of-range value */
int cisigma_set_option(cisigma_ctx *ctx, int key, double value);

/*
 * cisigma_apply -- sigma = H C (Eq. 5) for one vector.
 *   C, sigma   device arrays of ndet elements of dtype (CISIGMA_FP64 or
 *              CISIGMA_FP32), caller-owned, contiguous, in the vector order
 *              above.  They must not overlap (EINVAL).  sigma is overwritten.
 *   stream     hipStream_t or NULL.  The call only enqueues work: it returns
 *              before the result is ready; synchronise the stream to read it.
 * FP32 computes in FP32 (MFMA with FP32 accumulation); FP64 in FP64.
 * The first call for a dtype allocates that dtype's workspace (synchronous).
 * With CISIGMA_OPT_SPIN_PARITY p != 0 the caller guarantees
 * C(Ib, Ia) = p C(Ia, Ib); the beta-beta part is then taken as p times the
 * transpose of the alpha-alpha part (exact for such C; for any
 * other C the result is sigma_aa(C) + sigma_ab(C) + sigma_bb(p C^T)).
 */
int cisigma_apply(cisigma_ctx *ctx, const void *C, void *sigma, int dtype, void *stream);

/*
 * cisigma_apply_noalloc -- cisigma_apply for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same sigma = H C, with the same arguments,
 * ordering and asynchrony, and the same kernels, but the sigma workspace is
 * carved from a static device array of 64 MiB that the library holds on every
 * GPU it runs on until the process ends; the call makes no hipMalloc, hipFree
 * or other allocating call and no memset (it clears what must start at zero
 * with kernels).  Options act as for cisigma_apply except CISIGMA_OPT_PROFILE,
 * CISIGMA_OPT_OVERLAP and CISIGMA_OPT_GRAPH, which it ignores.
 *   Limit: the four padded layout copies of the space must fit in the 64 MiB
 *   (about 16 M elements FP32, 8 M FP64: CAS(12,12) and smaller in either
 *   precision); the materialised same-spin rows take what is left (column
 *   chunks), and when less than one 64-column chunk is left the same-spin parts
 *   run on the atomic kernels.  Larger spaces: EUNSUPPORTED, with the bytes
 *   needed in cisigma_last_error.
 *   The current device must be the one cisigma_init ran on (EINVAL otherwise).
 * Every call on a GPU shares that GPU's one array, whichever context makes it:
 * calls that overlap in time on one GPU (other streams, other host threads)
 * race on it and give wrong results.  Order them on one stream, or synchronise.
 */
int cisigma_apply_noalloc(cisigma_ctx *ctx, const void *C, void *sigma, int dtype, void *stream);

/*
 * cisigma_hmat_block -- Hamiltonian matrix elements between determinants of
 * the space (Eq. 6 with the string operators of Eq. 7: the Slater-Condon
 * rules): out[i * m + j] = H(rows[i], cols[j]) for vector indices rows[0..n)
 * and cols[0..m) (the order of cisigma_layout / cisigma_address).
 *   rows, cols  host int64 arrays; out host double[n * m], written.
 * Synchronous, evaluated on the host (for small blocks: a P-space, tests).
 * EINVAL for an index outside [0, ndet) or NULL arrays with n, m > 0.
 */
int cisigma_hmat_block(cisigma_ctx *ctx, int n, const int64_t *rows, int m, const int64_t *cols, double *out);

/*
 * cisigma_autotune -- picks the launch parameters of cisigma_apply for this
 * space and dtype by timing them (Sec. 3.3: the batches of the GAS partition;
 * here their order on one GPU): for each knob in turn, every candidate value
 * is set and reps applies of a fixed synthetic vector are timed with HIP
 * events; the fastest value stays set.  Knobs: the width of the owner-computes
 * units (CISIGMA_OPT_UNIT_COLS: the LDS, 16384, 8192, 4096 columns; the unit
 * tables are rebuilt for each), their launch order (most source tiles per row
 * first, alpha-type order, most total work first, heavy and light alternating)
 * and the column split of the same-spin pair-product kernel of spaces with
 * several types.  Results do not depend on the knobs beyond rounding order.
 *   dtype       CISIGMA_FP32 or CISIGMA_FP64: the precision tuned
 *   reps        timed applies per candidate, 1..100
 *   report      host char[report_len] (may be NULL when report_len = 0): one
 *               line per timing and per choice, NUL-terminated, truncated
 * Synchronous; allocates two vectors for the duration of the call; drops the
 * captured apply graphs.  EINVAL for bad arguments.
 */
int cisigma_autotune(cisigma_ctx *ctx, int dtype, int reps, char *report, int report_len);

/*
 * cisigma_hdiag -- diagonal H_II into the device array hdiag[ndet] (FP64),
 * asynchronously on stream: the diagonal of H that step (2) of the Davidson
 * iteration of Sec. 3.3 divides the residual by (the preconditioner), from the
 * Slater-Condon rules of Eq. 6 with I = J.  hdiag is caller-owned device
 * memory; EINVAL for a NULL context or array.
 */
int cisigma_hdiag(cisigma_ctx *ctx, double *hdiag, void *stream);

/*
 * cisigma_set_log -- JSON-lines log of cisigma_davidson: when path is a
 * non-empty string, every later Davidson call appends to that file one line per
 * iteration, {"call": c, "iteration": k, "dim": m, "precision": "fp64"|"mixed",
 * "energies": [...], "residuals": [...], "sigma_fp32": n, "sigma_fp64": n,
 * "seconds": t}, and one per FP64 refinement of the mixed mode (key
 * "refinement", energies = FP64 Rayleigh quotients, residuals = FP64 residual
 * norms).  NULL or "" stops logging.  The path is copied; the file is opened
 * and closed by each Davidson call.  EINVAL for a NULL context.
 */
int cisigma_set_log(cisigma_ctx *ctx, const char *path);

/*
 * cisigma_davidson -- lowest nroots eigenpairs of H (Sec. 3.3).
 *   nroots     1..64 (and <= ndet).
 *   tol        energy convergence threshold |delta E| between iterations.
 *   energies   host double[nroots], ascending.
 *   vecs       NULL, or caller-owned device array [nroots][ndet] of FP64
 *              (plain mode) or FP32 (mixed mode) receiving the eigenvectors.
 *   stats      NULL or statistics out.
 * Synchronous; runs on the context's own stream.  Returns ENOCONV when
 * max_iter is reached (energies and vectors are the last Ritz values).
 * In mixed mode (CISIGMA_OPT_PRECISION = CISIGMA_FP32) basis vectors and
 * sigma builds are FP32 while the projected matrix, orthogonalisation and
 * residual norms accumulate in FP64; when the FP32 iteration meets the test
 * (and every REFINE_EVERY iterations if that option is nonzero) the Ritz
 * vectors get an FP64 sigma, convergence is judged on their FP64 residuals,
 * and the returned energies are FP64 Rayleigh quotients <x|H x>/<x|x>.
 * With CISIGMA_OPT_SPIN_PARITY p != 0 the roots are the lowest of the sector
 * C(Ib, Ia) = p C(Ia, Ib): guesses are the combinations
 * (|Ia Ib> + p |Ib Ia>)/sqrt(2) (or |Ia Ia> for p = +1) of the lowest
 * diagonal elements, and every correction vector is projected onto the
 * sector.
 */
int cisigma_davidson(cisigma_ctx *ctx, int nroots, double tol, double *energies, void *vecs,
                     cisigma_stats *stats);

/*
 * cisigma_rdm -- spin-summed one- and two-particle density matrices of C (the
 * densities of the orbital step, Sec. 2.2 and Sec. 3.4), normalised by <C|C>:
 *     rdm1[p*n + q]               = sum_s <C|a+_ps a_qs|C> / <C|C>
 *     rdm2[((p*n + q)*n + r)*n + s] = sum_(s,t) <C|a+_ps a+_rt a_st a_qs|C> / <C|C>
 * (chemists' order: the energy is sum h_pq rdm1_pq + 1/2 sum (pq|rs) rdm2_pqrs).
 *   C          device vector of ndet elements of dtype (CISIGMA_FP64 or
 *              CISIGMA_FP32; FP32 multiplies in FP32 and sums the per-workgroup
 *              partials in FP64), caller-owned, in the vector order above.
 *   rdm1, rdm2 caller-owned device FP64 arrays of n^2 and n^4 elements,
 *              overwritten.  A zero vector gives NaN.
 *   stream     hipStream_t or NULL; asynchronous like cisigma_apply.
 * Built for one-block (CAS) spaces with norb <= 16 whose alpha-major row fits
 * the 160 KB LDS with the product tile (EUNSUPPORTED otherwise).  The first
 * call allocates a partial-sum buffer (~80 MB at norb = 16) and the dtype's
 * sigma workspace.
 */
int cisigma_rdm(cisigma_ctx *ctx, const void *C, int dtype, double *rdm1, double *rdm2, void *stream);

/*
 * cisigma_pass_times -- with CISIGMA_OPT_PROFILE set, every cisigma_apply
 * records a HIP event pair around each pass on the stream it runs on.  This
 * call synchronises those events and writes the summed milliseconds of each
 * pass since profiling was (re)enabled into ms[CISIGMA_NPASS] and the number
 * of profiled apply calls into *ncalls.  EINVAL when profiling is off.
 */
int cisigma_pass_times(cisigma_ctx *ctx, double *ms, int *ncalls);

/*
 * cisigma_last_path -- which kernels the most recent cisigma_apply of dtype
 * used, as CISIGMA_PATH_* flags in *flags (0 before any apply).  One-block
 * (CAS) and GAS spaces, with or without point-group symmetry, normally take
 * the materialised same-spin form; sigma_3 takes an owner-computes kernel
 * except with point-group symmetry.  Shapes outside the fast kernels' range,
 * spaces whose stored rows do not fit in memory, and CISIGMA_OPT_SIGMA_PATH = 1
 * use the general scatter kernels (flag clear).
 */
#define CISIGMA_PATH_AB_OWNER 1          /* sigma_3 by the owner-computes kernel (no global atomics) */
#define CISIGMA_PATH_SS_MATERIALISED 2   /* same-spin parts by materialised pair products + gather */
#define CISIGMA_PATH_AB_SHARED_CU 4      /* sigma_3 by the one-block owner kernel in its one-W-tile form, two
                                            workgroups per compute unit (FP32, where two fit) */
int cisigma_last_path(const cisigma_ctx *ctx, int dtype, int *flags);

/*
 * cisigma_last_shape -- the compiled shape of the owner-computes sigma_3
 * kernel (the alpha-beta part of Eq. 8) that the most recent cisigma_apply of
 * dtype launched, for tests that must know which variant ran:
 *   shape[0]  k steps of gathered alpha rows (4 rows each)
 *   shape[1]  16-row blocks of orbital pairs
 *   shape[2]  scatter-plan entries per lane and tile
 *   shape[3]  0: no owner-computes kernel ran (general kernel); 1: one-block
 *             kernel with the own row in a k step; 2: one-block kernel with the
 *             own row as the rank-1 start of the accumulators; 3: units of
 *             the GAS form (four waves); 4: units of a one-block space with
 *             its sigma row split, eight-wave form (FP32); 5: units of the GAS
 *             form, eight waves (FP32 with C below 4 GB)
 * shape is a host int[4], written.  EINVAL for NULL arguments or a bad dtype.
 */
int cisigma_last_shape(const cisigma_ctx *ctx, int dtype, int *shape);

/* message of the most recent failure on ctx (never NULL) */
const char *cisigma_last_error(const cisigma_ctx *ctx);

/* static description of a status code (never NULL) */
const char *cisigma_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* CISIGMA_H */
