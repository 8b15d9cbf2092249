// hmat.hip -- Hamiltonian matrix elements between individual determinants
// (host code): the Slater-Condon rules of Eq. 6, with the one-electron
// operators of Eq. 7 written on the alpha and beta strings.  They serve the
// Davidson P-space (the exact block of H over the determinants with the lowest
// diagonal elements: initial guess and preconditioner) and cisigma_hmat_block.
//
// Conventions: real orbitals, chemists' integrals (pq|rs); a determinant is
// the alpha string followed by the beta string, creators in ascending orbital
// order, so an operator on one spin's string takes the sign
// (-1)^(occupied orbitals of that string below it) and number-conserving
// pairs on the beta string take no sign from the alpha string.
#include "internal.h"

#include <algorithm>

namespace cis {
namespace {

inline int below_sign(uint32_t bits, int orb) {
    return (__builtin_popcount(bits & ((1u << orb) - 1u)) & 1) ? -1 : 1;
}

// sign of a+_p a_q |bits> (q occupied; p empty once q is removed)
inline int hop_sign(uint32_t bits, int p, int q) {
    const int s = below_sign(bits, q);
    return s * below_sign(bits & ~(1u << q), p);
}

struct Rules {
    int n;
    const double *h, *g;
    double eri(int p, int q, int r, int s) const { return g[((size_t(p) * n + q) * n + r) * n + s]; }

    double diagonal(uint32_t a, uint32_t b) const {
        double e = 0;
        for (uint32_t x = a; x; x &= x - 1) {
            const int p = __builtin_ctz(x);
            e += h[p * n + p];
            for (uint32_t y = a; y; y &= y - 1) {
                const int q = __builtin_ctz(y);
                e += 0.5 * (eri(p, p, q, q) - eri(p, q, q, p));
            }
            for (uint32_t y = b; y; y &= y - 1) {
                const int q = __builtin_ctz(y);
                e += eri(p, p, q, q);
            }
        }
        for (uint32_t x = b; x; x &= x - 1) {
            const int p = __builtin_ctz(x);
            e += h[p * n + p];
            for (uint32_t y = b; y; y &= y - 1) {
                const int q = __builtin_ctz(y);
                e += 0.5 * (eri(p, p, q, q) - eri(p, q, q, p));
            }
        }
        return e;
    }

    // <x1 o|H|x2 o>, x1 = a+_p a_q x2 on one spin, o the unchanged other string
    double single(uint32_t x1, uint32_t x2, uint32_t o) const {
        const int p = __builtin_ctz(x1 & ~x2), q = __builtin_ctz(x2 & ~x1);
        double v = h[p * n + q];
        for (uint32_t y = x2; y; y &= y - 1) {
            const int r = __builtin_ctz(y);
            v += eri(p, q, r, r) - eri(p, r, r, q);
        }
        for (uint32_t y = o; y; y &= y - 1) {
            const int r = __builtin_ctz(y);
            v += eri(p, q, r, r);
        }
        return hop_sign(x2, p, q) * v;
    }

    // same-spin double: x1 = a+_p1 a+_p2 a_q2 a_q1 x2 (p1 < p2, q1 < q2)
    double same_double(uint32_t x1, uint32_t x2) const {
        const uint32_t cr = x1 & ~x2, an = x2 & ~x1;
        const int p1 = __builtin_ctz(cr), p2 = 31 - __builtin_clz(cr);
        const int q1 = __builtin_ctz(an), q2 = 31 - __builtin_clz(an);
        uint32_t t = x2;
        int s = below_sign(t, q1);
        t &= ~(1u << q1);
        s *= below_sign(t, q2);
        t &= ~(1u << q2);
        s *= below_sign(t, p2);
        t |= 1u << p2;
        s *= below_sign(t, p1);
        return s * (eri(p1, q1, p2, q2) - eri(p1, q2, p2, q1));
    }

    double element(uint32_t a1, uint32_t b1, uint32_t a2, uint32_t b2) const {
        const int da = __builtin_popcount(a1 ^ a2), db = __builtin_popcount(b1 ^ b2);   // twice the differences
        if (da + db > 4) return 0.0;
        if (da == 0 && db == 0) return diagonal(a1, b1);
        if (da == 2 && db == 0) return single(a1, a2, b1);
        if (da == 0 && db == 2) return single(b1, b2, a1);
        if (da == 4) return same_double(a1, a2);
        if (db == 4) return same_double(b1, b2);
        // one alpha and one beta excitation: (pq|rs) times both hop signs
        const int p = __builtin_ctz(a1 & ~a2), q = __builtin_ctz(a2 & ~a1);
        const int r = __builtin_ctz(b1 & ~b2), s = __builtin_ctz(b2 & ~b1);
        return hop_sign(a2, p, q) * hop_sign(b2, r, s) * eri(p, q, r, s);
    }
};

}  // namespace

bool det_strings(const cisigma_ctx *c, int64_t idx, const std::vector<uint32_t> &astr,
                 const std::vector<uint32_t> &bstr, uint32_t *a, uint32_t *b) {
    const auto &L = c->lay;
    if (idx < 0 || idx >= L.ndet) return false;
    const int blk = int(std::upper_bound(L.blk_off.begin(), L.blk_off.begin() + L.nblk, idx) - L.blk_off.begin()) - 1;
    if (blk < 0) return false;
    const int ta = L.blk_a[blk], tb = L.blk_b[blk];
    const int64_t ncol = c->sp[1].tcount[tb];
    const int64_t rel = idx - L.blk_off[blk];
    *a = astr[size_t(c->sp[0].tstart[ta] + rel / ncol)];
    *b = bstr[size_t(c->sp[1].tstart[tb] + rel % ncol)];
    return true;
}

double hmat_element(const cisigma_ctx *c, uint32_t a1, uint32_t b1, uint32_t a2, uint32_t b2) {
    const Rules R{c->n, c->h.data(), c->g.data()};
    return R.element(a1, b1, a2, b2);
}

}  // namespace cis
