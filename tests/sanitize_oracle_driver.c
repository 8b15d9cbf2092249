/* Runs the oracle (oracle/oracle.c, compiled into this program) on a space
 * read from stdin, for the AddressSanitizer / UndefinedBehaviorSanitizer
 * build of tests/test_sanitizers.py.  Input: norb na nb ngas, then ngas
 * values each of gas_norb, min_cum, max_cum, then h (norb^2), eri (norb^4)
 * and C (ndet, after the space is built).  Output: ndet, sigma, hdiag, the
 * one- and two-particle density matrices and H(i, j) for a few pairs. */
#include <stdio.h>
#include "../oracle/oracle.c"

static int rd(double *x) { return scanf("%lf", x) == 1; }

int main(void) {
    int norb, na, nb, ngas;
    if (scanf("%d %d %d %d", &norb, &na, &nb, &ngas) != 4 || ngas < 1 || ngas > 8) return 2;
    int gn[8], mn[8], mx[8];
    for (int g = 0; g < ngas; ++g) if (scanf("%d", &gn[g]) != 1) return 2;
    for (int g = 0; g < ngas; ++g) if (scanf("%d", &mn[g]) != 1) return 2;
    for (int g = 0; g < ngas; ++g) if (scanf("%d", &mx[g]) != 1) return 2;
    const size_t n2 = (size_t)norb * norb;
    double *h = malloc(n2 * sizeof(double)), *eri = malloc(n2 * n2 * sizeof(double));
    for (size_t i = 0; i < n2; ++i) if (!rd(&h[i])) return 2;
    for (size_t i = 0; i < n2 * n2; ++i) if (!rd(&eri[i])) return 2;
    or_space *S = or_create(norb, na, nb, ngas, gn, mn, mx, h, eri);
    if (!S) return 3;
    const int64_t nd = or_ndet(S);
    double *C = malloc(nd * sizeof(double)), *sig = malloc(nd * sizeof(double)), *hd = malloc(nd * sizeof(double));
    double *r1 = malloc(n2 * sizeof(double)), *r2 = malloc(n2 * n2 * sizeof(double));
    for (int64_t i = 0; i < nd; ++i) if (!rd(&C[i])) return 2;
    or_sigma(S, C, sig);
    or_hdiag(S, hd);
    or_rdm(S, C, r1, r2);
    printf("%lld\n", (long long)nd);
    for (int64_t i = 0; i < nd; ++i) printf("%.17g\n", sig[i]);
    for (int64_t i = 0; i < nd; ++i) printf("%.17g\n", hd[i]);
    for (size_t i = 0; i < n2; ++i) printf("%.17g\n", r1[i]);
    for (size_t i = 0; i < n2 * n2; ++i) printf("%.17g\n", r2[i]);
    for (int64_t i = 0; i < nd; i += 7) printf("%.17g\n", or_h_elem(S, i, (i * 13 + 5) % nd));
    or_free(S);
    free(C); free(sig); free(hd); free(r1); free(r2); free(h); free(eri);
    return 0;
}
