// Reads n and an n x n symmetric matrix (row-major) from stdin; prints the
// convergence flag, then the eigenvalues and the eigenvector matrix of
// cis::sym_eig (the host eigensolver of the Davidson driver).
#include <cstdio>
#include <vector>

#include "symeig.h"

int main() {
    int n;
    if (std::scanf("%d", &n) != 1 || n < 0) return 1;
    std::vector<double> A(size_t(n) * n), w, V;
    for (auto &x : A)
        if (std::scanf("%lf", &x) != 1) return 1;
    const bool ok = cis::sym_eig(A, n, w, V);
    std::printf("%d\n", ok ? 1 : 0);
    for (double x : w) std::printf("%.17g\n", x);
    for (double x : V) std::printf("%.17g\n", x);
    return 0;
}
