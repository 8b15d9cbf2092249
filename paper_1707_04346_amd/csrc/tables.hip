// tables.hip -- integer string tables built on the device (bit-exact).
//
// * strings of each occupation type (Sec. 3.1, Eq. 9 without the symmetry
//   label): a string of type T is a product of one sub-string per GAS space;
//   its rank inside the type is a mixed-radix number whose digits are the
//   colex ranks of the sub-strings, space 0 the fastest digit.  This is the
//   ascending-bitmask order of the strings of a type.
// * single-excitation ("connection", Sec. 3.1) lists: for string I, every
//   J = a^+_l a_k I with k occupied and l empty, with the sign of the
//   operator string (Eq. 2 ordering) -- the E_kl lists of Sec. 3.3.
// * pair lists: for every (nel-2)-electron string K and every pair of empty
//   orbitals j < l of K, the string J = a^+_j a^+_l K and its sign; these
//   drive the same-spin two-electron part of sigma (sigma_1 / sigma_2 of Eq. 8).
#include "internal.h"

#include <algorithm>
#include <vector>

namespace cis {
namespace {

__constant__ uint32_t c_binom[33][33];

__device__ __forceinline__ int popc(uint32_t x) { return __popc(x); }

// colex rank of a sub-string (bit positions relative to the space start)
__device__ __forceinline__ uint32_t colex_rank(uint32_t sub) {
    uint32_t r = 0;
    int i = 1;
    while (sub) {
        int p = __ffs(sub) - 1;
        r += c_binom[p][i];
        ++i;
        sub &= sub - 1;
    }
    return r;
}

// string of colex rank r with k electrons among m positions
__device__ __forceinline__ uint32_t colex_unrank(uint32_t r, int k, int m) {
    uint32_t s = 0;
    int hi = m - 1;
    for (int i = k; i >= 1; --i) {
        int c = hi;
        while (c >= i && c_binom[c][i] > r) --c;
        // c_binom[c][i] <= r (c >= i-1; c_binom[i-1][i] = 0)
        s |= 1u << c;
        r -= c_binom[c][i];
        hi = c - 1;
    }
    return s;
}

struct TypeView {
    const uint64_t *key;     // GAS type keys (sorted)
    const int *start;        // first raw index of each GAS type
    const uint32_t *radix;
    int ntype;
    const int *remap;        // raw index -> string index (spatial symmetry), or nullptr
};

// index of string x in the spin's string list, or -1
__device__ int string_index(uint32_t x, const GasDesc &g, const TypeView &tv) {
    uint64_t key = 0;
    for (int s = 0; s < g.ngas; ++s) key += uint64_t(popc(x & g.mask[s])) * g.keymul[s];
    int lo = 0, hi = tv.ntype - 1, t = -1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        uint64_t k = tv.key[mid];
        if (k == key) { t = mid; break; }
        if (k < key) lo = mid + 1; else hi = mid - 1;
    }
    if (t < 0) return -1;
    uint32_t r = 0;
    for (int s = 0; s < g.ngas; ++s) r += colex_rank((x & g.mask[s]) >> g.first[s]) * tv.radix[t * g.ngas + s];
    const int raw = tv.start[t] + int(r);
    return tv.remap ? tv.remap[raw] : raw;
}

__global__ void k_unrank(uint32_t *str, int *stype, int t, int start, int count, GasDesc g, const int *occ,
                         const uint32_t *radix_t) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count) return;
    uint32_t rem = uint32_t(r), x = 0;
    for (int s = 0; s < g.ngas; ++s) {
        int m = popc(g.mask[s]);
        uint32_t base = c_binom[m][occ[s]];
        uint32_t d = rem % base;
        rem /= base;
        x |= colex_unrank(d, occ[s], m) << g.first[s];
    }
    (void)radix_t;
    str[start + r] = x;
    stype[start + r] = t;
}

// entries per string: nel * (n - nel); thread per (string, entry)
__global__ void k_build_exc(uint32_t *exc, const uint32_t *str, int nstr, int nel, GasDesc g, TypeView tv) {
    int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int nvir = g.n - nel;
    int per = nel * nvir;
    if (per == 0 || tid >= int64_t(nstr) * per) return;
    int I = int(tid / per);
    int e = int(tid % per);
    int ko = e / nvir, lv = e % nvir;
    uint32_t x = str[I];
    uint32_t full = (g.n >= 32) ? 0xFFFFFFFFu : ((1u << g.n) - 1u);
    uint32_t occ = x, vir = full & ~x;
    for (int i = 0; i < ko; ++i) occ &= occ - 1;
    for (int i = 0; i < lv; ++i) vir &= vir - 1;
    int k = __ffs(occ) - 1, l = __ffs(vir) - 1;
    uint32_t y = (x & ~(1u << k)) | (1u << l);
    int J = string_index(y, g, tv);
    uint32_t out = kExcNone;
    if (J >= 0) {
        int lo = k < l ? k : l, hi = k < l ? l : k;
        uint32_t between = (hi - lo > 1) ? (((hi >= 32) ? 0xFFFFFFFFu : ((1u << hi) - 1u)) & ~((1u << (lo + 1)) - 1u)) : 0u;
        bool neg = popc(x & between) & 1;
        out = exc_pack(uint32_t(J), k, l, neg);
    }
    exc[tid] = out;
}

// pair lists: thread per (K, pair entry)
__global__ void k_build_pairs(uint32_t *pairs, int nK, int kel, int npv, GasDesc g, TypeView tv) {
    int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tid >= int64_t(nK) * npv) return;
    int K = int(tid / npv);
    int e = int(tid % npv);
    uint32_t kb = colex_unrank(uint32_t(K), kel, g.n);
    uint32_t full = (g.n >= 32) ? 0xFFFFFFFFu : ((1u << g.n) - 1u);
    uint32_t vir = full & ~kb;
    int nv = popc(vir);
    // e -> (a < b) over the empty orbitals of K, a-major
    int a = 0, rem = e;
    while (rem >= nv - 1 - a) { rem -= nv - 1 - a; ++a; }
    int b = a + 1 + rem;
    uint32_t v = vir;
    for (int i = 0; i < a; ++i) v &= v - 1;
    int j = __ffs(v) - 1;
    for (int i = a; i < b; ++i) v &= v - 1;
    int l = __ffs(v) - 1;
    uint32_t y = kb | (1u << j) | (1u << l);
    int J = string_index(y, g, tv);
    uint32_t out = kPairNone;
    if (J >= 0) {
        // sign of a^+_j a^+_l |K>: occupied orbitals of K below l, plus below j
        int s = popc(kb & ((1u << l) - 1u)) + popc(kb & ((1u << j) - 1u));
        out = (uint32_t(J) << 11) | (uint32_t(pair_gt(l, j)) << 1) | uint32_t(s & 1);
    }
    pairs[tid] = out;
}

// inverse of the pair lists: for string I and each occupied pair p < r of I
// (lexicographic), the row K*npv + e of the pair-list entry that produces I
// from K = I - p - r, or -1 when I is not in the list of K.
__global__ void k_build_pair_inv(int *inv, const uint32_t *str, int nstr, int nel, int npv, int n) {
    const int per = nel * (nel - 1) / 2;
    int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (per == 0 || tid >= int64_t(nstr) * per) return;
    const int I = int(tid / per);
    int slot = int(tid % per);
    const uint32_t x = str[I];
    // slot -> (a < b) over the occupied orbitals of I
    int a = 0, rem = slot;
    while (rem >= nel - 1 - a) { rem -= nel - 1 - a; ++a; }
    const int b = a + 1 + rem;
    uint32_t o = x;
    for (int i = 0; i < a; ++i) o &= o - 1;
    const int p = __ffs(o) - 1;
    for (int i = a; i < b; ++i) o &= o - 1;
    const int r = __ffs(o) - 1;
    const uint32_t kb = x & ~(1u << p) & ~(1u << r);
    // colex rank of K among (nel-2)-electron strings of n orbitals
    uint32_t K = colex_rank(kb);
    // positions of p and r among the empty orbitals of K
    const int nv = n - (nel - 2);
    const int ap = p - popc(kb & ((1u << p) - 1u));
    const int ar = r - popc(kb & ((1u << r) - 1u));
    const int e = ap * (nv - 1) - ap * (ap - 1) / 2 + (ar - ap - 1);
    (void)nv;
    inv[tid] = int(K) * npv + e;
}

// A_s[I] = sum_{p in I} h_pp + 1/2 sum_{p,q in I} ((pp|qq) - (pq|qp))
__global__ void k_adiag(double *out, const uint32_t *str, int nstr, const double *h, const double *g4, int n) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nstr) return;
    uint32_t x = str[I];
    double e = 0.0;
    for (uint32_t a = x; a; a &= a - 1) {
        int p = __ffs(a) - 1;
        e += h[p * n + p];
        for (uint32_t b = x; b; b &= b - 1) {
            int q = __ffs(b) - 1;
            size_t pq = size_t(p) * n + q;
            e += 0.5 * (g4[(size_t(p) * n + p) * n * n + size_t(q) * n + q] - g4[pq * n * n + size_t(q) * n + p]);
        }
    }
    out[I] = e;
}

bool g_binom_ready = false;

}  // namespace

static hipError_t upload_binom() {
    if (g_binom_ready) return hipSuccess;
    uint32_t b[33][33];
    for (int m = 0; m <= 32; ++m)
        for (int k = 0; k <= 32; ++k) {
            if (k > m) { b[m][k] = 0; continue; }
            uint64_t c = 1;
            for (int i = 0; i < k; ++i) c = c * uint64_t(m - i) / uint64_t(i + 1);
            b[m][k] = uint32_t(c);
        }
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_binom), b, sizeof(b));
    if (e == hipSuccess) g_binom_ready = true;
    return e;
}

#define CIS_TRY(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return e_; } while (0)

static uint64_t binom_host(int m, int k) {
    if (k < 0 || k > m) return 0;
    uint64_t c = 1;
    for (int i = 0; i < k; ++i) c = c * uint64_t(m - i) / uint64_t(i + 1);
    return c;
}

hipError_t build_string_tables(cisigma_ctx *ctx, int spin) {
    CIS_TRY(upload_binom());
    SpinTables &T = ctx->sp[spin];
    const GasDesc &g = ctx->gas;
    int G = g.ngas;
    // host-side per-GAS-type radix of the raw rank
    std::vector<uint32_t> radix(size_t(std::max(T.ngtype, 1)) * G, 0);
    for (int t = 0; t < T.ngtype; ++t) {
        uint64_t r = 1;
        for (int s = 0; s < G; ++s) {
            radix[size_t(t) * G + s] = uint32_t(r);
            r *= binom_host(__builtin_popcount(g.mask[s]), T.gtocc[size_t(t) * G + s]);
        }
    }
    size_t ns = size_t(T.nstr > 0 ? T.nstr : 1);
    CIS_TRY(hipMalloc(&T.d_str, ns * sizeof(uint32_t)));
    CIS_TRY(hipMalloc(&T.d_stype, ns * sizeof(int)));
    CIS_TRY(hipMalloc(&T.d_gkey, size_t(T.ngtype > 0 ? T.ngtype : 1) * sizeof(uint64_t)));
    CIS_TRY(hipMalloc(&T.d_graw, size_t(T.ngtype + 1) * sizeof(int)));
    CIS_TRY(hipMalloc(&T.d_radix, radix.size() * sizeof(uint32_t)));
    if (T.ngtype > 0) CIS_TRY(hipMemcpy(T.d_gkey, T.gkey.data(), T.ngtype * sizeof(uint64_t), hipMemcpyHostToDevice));
    CIS_TRY(hipMemcpy(T.d_graw, T.graw.data(), (T.ngtype + 1) * sizeof(int), hipMemcpyHostToDevice));
    CIS_TRY(hipMemcpy(T.d_radix, radix.data(), radix.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    int *d_occ = nullptr;
    CIS_TRY(hipMalloc(&d_occ, size_t(T.ntype > 0 ? T.ntype : 1) * G * sizeof(int)));
    if (!ctx->sym) {
        // the strings of each type by their mixed-radix rank on the device
        CIS_TRY(hipMemcpy(d_occ, T.tocc.data(), T.tocc.size() * sizeof(int), hipMemcpyHostToDevice));
        for (int t = 0; t < T.ntype; ++t) {
            int cnt = T.tcount[t];
            if (cnt == 0) continue;
            hipLaunchKernelGGL(k_unrank, dim3((cnt + 255) / 256), dim3(256), 0, ctx->stream, T.d_str, T.d_stype, t,
                               T.tstart[t], cnt, g, d_occ + t * G, T.d_radix + t * G);
            CIS_TRY(hipGetLastError());
        }
    } else {
        // spatial symmetry: the strings of each (GAS type, irrep) type, in order, from the
        // host enumeration of the raw strings, and the raw -> string index map
        std::vector<uint32_t> str(ns, 0);
        std::vector<int> stype(ns, 0);
        for (int gt = 0; gt < T.ngtype; ++gt) {
            std::vector<std::vector<uint32_t>> sub(G);
            for (int s2 = 0; s2 < G; ++s2) {
                const int m = __builtin_popcount(g.mask[s2]), k = T.gtocc[size_t(gt) * G + s2];
                uint64_t x = (uint64_t(1) << k) - 1;
                for (uint64_t c = 0; c < binom_host(m, k); ++c) {
                    sub[s2].push_back(uint32_t(x) << g.first[s2]);
                    if (x == 0) break;
                    const uint64_t lo = x & (~x + 1), r = x + lo;
                    x = (((r ^ x) >> 2) / lo) | r;
                }
            }
            for (int raw = T.graw[gt]; raw < T.graw[gt + 1]; ++raw) {
                const int idx = T.remap[raw];
                if (idx < 0) continue;
                uint32_t rem = uint32_t(raw - T.graw[gt]), x = 0;
                for (int s2 = 0; s2 < G; ++s2) {
                    const uint32_t base = uint32_t(sub[s2].size());
                    x |= sub[s2][rem % base];
                    rem /= base;
                }
                str[idx] = x;
            }
        }
        for (int t = 0; t < T.ntype; ++t)
            for (int i = T.tstart[t]; i < T.tstart[t + 1]; ++i) stype[i] = t;
        CIS_TRY(hipMemcpy(T.d_str, str.data(), size_t(T.nstr) * sizeof(uint32_t), hipMemcpyHostToDevice));
        CIS_TRY(hipMemcpy(T.d_stype, stype.data(), size_t(T.nstr) * sizeof(int), hipMemcpyHostToDevice));
        CIS_TRY(hipMalloc(&T.d_remap, std::max<size_t>(T.remap.size(), 1) * sizeof(int)));
        if (!T.remap.empty())
            CIS_TRY(hipMemcpy(T.d_remap, T.remap.data(), T.remap.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    TypeView tv{T.d_gkey, T.d_graw, T.d_radix, T.ngtype, T.d_remap};
    // single-excitation lists
    T.nexc = T.nel * (g.n - T.nel);
    if (T.nexc > 0 && T.nstr > 0) {
        int64_t tot = int64_t(T.nstr) * T.nexc;
        CIS_TRY(hipMalloc(&T.d_exc, size_t(tot) * sizeof(uint32_t)));
        hipLaunchKernelGGL(k_build_exc, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, ctx->stream, T.d_exc,
                           T.d_str, T.nstr, T.nel, g, tv);
        CIS_TRY(hipGetLastError());
    }
    // pair lists over (nel-2)-electron strings
    if (T.nel >= 2) {
        T.nK = int(binom_host(g.n, T.nel - 2));
        T.npv = int(binom_host(g.n - T.nel + 2, 2));
        int64_t tot = int64_t(T.nK) * T.npv;
        CIS_TRY(hipMalloc(&T.d_pairs, size_t(tot) * sizeof(uint32_t)));
        hipLaunchKernelGGL(k_build_pairs, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, ctx->stream, T.d_pairs,
                           T.nK, T.nel - 2, T.npv, g, tv);
        CIS_TRY(hipGetLastError());
    }
    // inverse pair table (the gather of the materialised same-spin path: at most
    // 64 occupied pairs per string)
    if (T.nel >= 2 && T.nel * (T.nel - 1) / 2 <= 64) {
        int per = T.nel * (T.nel - 1) / 2;
        int64_t tot = int64_t(T.nstr) * per;
        CIS_TRY(hipMalloc(&T.d_pair_inv, size_t(tot) * sizeof(int)));
        hipLaunchKernelGGL(k_build_pair_inv, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, ctx->stream,
                           T.d_pair_inv, T.d_str, T.nstr, T.nel, T.npv, g.n);
        CIS_TRY(hipGetLastError());
    }
    CIS_TRY(hipStreamSynchronize(ctx->stream));
    CIS_TRY(hipFree(d_occ));
    return hipSuccess;
}

hipError_t build_diag_tables(cisigma_ctx *ctx) {
    int n = ctx->n;
    double *d_h = nullptr, *d_g = nullptr;
    size_t n2 = size_t(n) * n;
    CIS_TRY(hipMalloc(&d_h, n2 * sizeof(double)));
    CIS_TRY(hipMalloc(&d_g, n2 * n2 * sizeof(double)));
    CIS_TRY(hipMemcpy(d_h, ctx->h.data(), n2 * sizeof(double), hipMemcpyHostToDevice));
    CIS_TRY(hipMemcpy(d_g, ctx->g.data(), n2 * n2 * sizeof(double), hipMemcpyHostToDevice));
    for (int s = 0; s < 2; ++s) {
        SpinTables &T = ctx->sp[s];
        CIS_TRY(hipMalloc(&T.d_adiag, size_t(T.nstr > 0 ? T.nstr : 1) * sizeof(double)));
        if (T.nstr > 0) {
            hipLaunchKernelGGL(k_adiag, dim3((T.nstr + 255) / 256), dim3(256), 0, ctx->stream, T.d_adiag, T.d_str,
                               T.nstr, d_h, d_g, n);
            CIS_TRY(hipGetLastError());
        }
    }
    CIS_TRY(hipStreamSynchronize(ctx->stream));
    CIS_TRY(hipFree(d_h));
    CIS_TRY(hipFree(d_g));
    return hipSuccess;
}

}  // namespace cis
