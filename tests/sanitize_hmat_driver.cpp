// Runs the library's host Slater-Condon rules (csrc/hmat.hip, compiled as
// host C++) on determinant pairs read from stdin, for the AddressSanitizer /
// UndefinedBehaviorSanitizer build of tests/test_sanitizers.py.  Input: norb,
// h (norb^2), eri (norb^4), npairs, then npairs lines "a1 b1 a2 b2" (string
// bitmasks).  Output: one H element per pair.
#include <cstdio>

#include "internal.h"

int main() {
    int n = 0;
    if (std::scanf("%d", &n) != 1 || n < 1 || n > 32) return 2;
    cisigma_ctx c;
    c.n = n;
    c.h.resize(size_t(n) * n);
    c.g.resize(size_t(n) * n * n * n);
    for (auto &x : c.h) if (std::scanf("%lf", &x) != 1) return 2;
    for (auto &x : c.g) if (std::scanf("%lf", &x) != 1) return 2;
    int np = 0;
    if (std::scanf("%d", &np) != 1 || np < 0) return 2;
    for (int i = 0; i < np; ++i) {
        unsigned a1, b1, a2, b2;
        if (std::scanf("%u %u %u %u", &a1, &b1, &a2, &b2) != 4) return 2;
        std::printf("%.17g\n", cis::hmat_element(&c, a1, b1, a2, b2));
    }
    return 0;
}
