// rdm.hip -- spin-summed one- and two-particle density matrices of a CI vector
// (the densities the orbital step of Sec. 2.2 and Sec. 3.4 consumes), for
// one-block (CAS) spaces of up to 16 orbitals.
//
// With D_rs(K) = <K|E_rs|C> = sum_J <K|E_rs|J> C_J (E_rs = E^a_rs + E^b_rs,
// Eq. 7) and the determinants K as a resolution of the identity,
//     <C|E_pq E_rs|C> = sum_K D_qp(K) D_rs(K),    <C|E_pq|C> = sum_K C_K D_pq(K),
// so the symmetric matrix M = [D; C] [D; C]^T (rows rs = r*n + s, then one row
// holding C itself) contains both products and <C|C>:
//     gamma_pq   = M[C, pq] / M[C, C],
//     Gamma_pqrs = M[qp, rs] / M[C, C] - d_qr gamma_ps,
// with Gamma in chemists' order (E = sum h gamma + 1/2 sum (pq|rs) Gamma).
//
// One workgroup per alpha string K_a at a time (grid-stride) keeps the row
// C(K_a, .) in LDS and builds D for NT beta strings K_b per tile:
//   alpha part: row (k, l) = sign * C(J_a, K_b) for each single alpha
//               excitation J_a = K_a - k + l (sign = <K_a|E_kl|J_a>);
//   beta part:  row (k, l) += sign * C(K_a, J_b) for each single beta
//               excitation J_b = K_b - k + l, read from the LDS row;
//   diagonal:   row (r, r) = (n^a_r + n^b_r) C(K),  last row = C(K).
// The tile's contribution D D^T goes to the matrix cores: the upper triangle
// of 16x16 blocks of M, split evenly over the eight waves, accumulated in
// registers across all tiles of the workgroup and written once per workgroup
// as FP64 partial sums, which a second kernel adds up.
#include "internal.h"
#include "mfma.h"

#include <algorithm>

namespace cis {
namespace {

constexpr int kRdmSlots = 20;   // block pairs per wave: ceil(153 / 8) for 17 row blocks
constexpr int kRdmMaxBlocks = 17;

template <typename T>
struct RdmArgs {
    const T *cp;                 // alpha-major padded C, row stride ld, padding columns zero
    const uint32_t *aexc, *bexc; // single-excitation lists of both spins
    const uint32_t *astr, *bstr; // string bitmasks
    double *part;                // [gridDim.x][npb][256] partial sums of the M blocks
    int n, Na, Nb, ld, anexc, bnexc, nb, npb;
};

template <typename T, int NT>
__global__ __launch_bounds__(512, 1) void k_rdm(RdmArgs<T> p) {
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    // D is stored with the columns of a tile permuted so that the k steps a lane
    // feeds to the matrix cores are contiguous: column c sits at
    // (c % 4) * KT + c / 4, and one lane's operand for all KT k steps is KT
    // consecutive elements (16-byte loads).  Rows are padded by 16 bytes.
    constexpr int KT = NT / 4;                             // k steps per tile
    constexpr int VE = 16 / int(sizeof(T));                // elements per 16-byte load
    constexpr int DS = NT + VE;                            // D row stride (elements)
    using V = typename M::vec_t;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *D = reinterpret_cast<T *>(smem_raw);                // [16 nb][DS]
    T *row = D + 16 * p.nb * DS;                           // [ld]: C(K_a, .)
    // what fills row r of D for this K_a: rowJ >= 0: alpha excitation J_a with
    // sign rowS; -1: zero; -2: C(K) itself; -3: diagonal row (k, k), rowS = k + 256 n^a_k
    int *rowJ = reinterpret_cast<int *>(row + p.ld);       // [16 nb]
    int *rowS = rowJ + 16 * p.nb;                          // [16 nb]
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = p.n, n2 = n * n, MR = 16 * p.nb;
    constexpr int RG = 512 / NT;                           // threads per tile column
    constexpr int KA = (64 + RG - 1) / RG;                 // single excitations per string <= 8 * 8 (n <= 16)
    constexpr int KB = KA;
    const int c = tid % NT, rg = tid / NT;
    const int cperm = (c % 4) * KT + c / 4;                // where column c is stored
    const int lfrag = (lane & 15) * DS + (lane >> 4) * KT; // this lane's operand inside a 16-row block

    // this wave's block pairs (bi <= bj), a contiguous run of the row-major
    // enumeration of the upper triangle, and their LDS fragment offsets
    const int per = (p.npb + 7) / 8;
    const int s0 = wave * per;
    int sbi[kRdmSlots], sbj[kRdmSlots];                    // block rows / columns of the slots
    int nslot = 0;
    {
        int bi = 0, bj = 0, q = 0;
        while (q < s0 && bi < p.nb) {                      // walk to pair s0
            if (++bj == p.nb) { ++bi; bj = bi; }
            ++q;
        }
#pragma unroll
        for (int s = 0; s < kRdmSlots; ++s) {
            const bool ok = s < per && s0 + s < p.npb;
            sbi[s] = ok ? bi : 0;
            sbj[s] = ok ? bj : 0;
            nslot += ok ? 1 : 0;
            if (ok && ++bj == p.nb) { ++bi; bj = bi; }
        }
    }
    acc_t acc[kRdmSlots];
#pragma unroll
    for (int s = 0; s < kRdmSlots; ++s) acc[s] = acc_t{0, 0, 0, 0};
    // partial sums of this workgroup: block pair s0 + s, element (row, col) at row*16 + col
    double *out = p.part + int64_t(blockIdx.x) * p.npb * 256;
    bool first = true;

    for (int Ka = blockIdx.x; Ka < p.Na; Ka += gridDim.x) {
        const T *crow = p.cp + int64_t(Ka) * p.ld;
        const uint32_t xa = p.astr[Ka];
        for (int c = tid; c < p.ld; c += 512) row[c] = crow[c];
        for (int r = tid; r < MR; r += 512) {
            int kind = r == n2 ? -2 : -1, aux = 0;
            if (r < n2 && r / n == r % n) {
                kind = -3;
                aux = r / n + 256 * int((xa >> (r / n)) & 1u);
            }
            rowJ[r] = kind;
            rowS[r] = aux;
        }
        __syncthreads();
        for (int e = tid; e < p.anexc; e += 512) {
            const uint32_t w = p.aexc[int64_t(Ka) * p.anexc + e];
            if (w == kExcNone) continue;
            const int k = (w >> 6) & 31, l = (w >> 1) & 31;
            rowJ[k * n + l] = int(w >> 11);
            rowS[k * n + l] = (w & 1) ? -1 : 1;
        }
        // this thread's column c of every tile, its alpha entries a = rg + RG i
        // (source offset, target row, sign) and beta entries e = rg + RG i
        uint32_t asrc[KA];
        int adst[KA];
        T asgn[KA];
#pragma unroll
        for (int i = 0; i < KA; ++i) {
            const int a = rg + RG * i;
            const uint32_t w = a < p.anexc ? p.aexc[int64_t(Ka) * p.anexc + a] : kExcNone;
            adst[i] = w == kExcNone ? -1 : int(((w >> 6) & 31) * n + ((w >> 1) & 31));
            asrc[i] = w == kExcNone ? 0u : (w >> 11) * uint32_t(p.ld) + uint32_t(c);
            asgn[i] = (w & 1) ? T(-1) : T(1);
        }
        // operands of tile c0 in registers, those of the next tile in flight
        T aval[KA], anext[KA];
        uint32_t bw[KB], bnext[KB], bs, bsnext;
        auto fetch = [&](int t0, T (&av)[KA], uint32_t (&bv)[KB], uint32_t &bsv) {
            const int Kb = t0 + c;
#pragma unroll
            for (int i = 0; i < KA; ++i) av[i] = adst[i] >= 0 ? p.cp[asrc[i] + uint32_t(t0)] : T(0);
            const bool in = Kb < p.Nb;
#pragma unroll
            for (int i = 0; i < KB; ++i) {
                const int e = rg + RG * i;
                bv[i] = in && e < p.bnexc ? p.bexc[int64_t(Kb) * p.bnexc + e] : kExcNone;
            }
            bsv = in ? p.bstr[Kb] : 0u;
        };
        fetch(0, aval, bw, bs);
        // D starts at zero for this K_a; afterwards each tile rewrites the alpha,
        // diagonal and C rows and clears the cells of zero rows that the previous
        // tile's beta part wrote
        for (int i = tid; i < MR * DS; i += 512) D[i] = T(0);
        uint32_t bprev[KB];
#pragma unroll
        for (int i = 0; i < KB; ++i) bprev[i] = kExcNone;
        __syncthreads();
        for (int c0 = 0; c0 < p.ld; c0 += NT) {
            if (c0 + NT < p.ld) fetch(c0 + NT, anext, bnext, bsnext);
            const int Kb = c0 + c;
#pragma unroll
            for (int i = 0; i < KB; ++i) {
                const uint32_t w = bprev[i];
                if (w == kExcNone) continue;
                const int r = int(((w >> 6) & 31) * n + ((w >> 1) & 31));
                if (rowJ[r] == -1) D[r * DS + cperm] = T(0);
            }
            // diagonal rows (k, k) for orbitals k = rg, rg + RG, ... and the C row (k = n)
            for (int k = rg; k <= n; k += RG) {
                const int r = k < n ? k * n + k : n2;
                T v = row[Kb];
                if (k < n) v *= T((rowS[r] >> 8) + int((bs >> k) & 1u));
                D[r * DS + cperm] = v;
            }
            // alpha rows (padding columns of C are zero)
#pragma unroll
            for (int i = 0; i < KA; ++i)
                if (adst[i] >= 0) D[adst[i] * DS + cperm] = asgn[i] * aval[i];
            __syncthreads();
            // beta part: within a column the excitations have distinct (k, l),
            // so no two threads add to one cell
#pragma unroll
            for (int i = 0; i < KB; ++i) {
                const uint32_t w = bw[i];
                if (w == kExcNone) continue;
                const int k = (w >> 6) & 31, l = (w >> 1) & 31;
                const T u = row[w >> 11];
                D[(k * n + l) * DS + cperm] += (w & 1) ? -u : u;
            }
            __syncthreads();
            // M += D D^T over the tile's columns: per slot one operand of each
            // block (all KT k steps), the row operand reloaded only when the
            // block row changes, the next slot's column operand in flight
            {
                auto frag = [&](int blk, T (&f)[KT]) {
                    const V *src = reinterpret_cast<const V *>(D + 16 * blk * DS + lfrag);
#pragma unroll
                    for (int v = 0; v < KT / VE; ++v) {
                        const V x = src[v];
#pragma unroll
                        for (int e = 0; e < VE; ++e) f[v * VE + e] = x[e];
                    }
                };
                // slots in groups of SG: SG independent accumulation chains per k step
                constexpr int SG = sizeof(T) == 4 ? 2 : 1;
#pragma unroll
                for (int g0 = 0; g0 < kRdmSlots; g0 += SG) {
                    if (g0 < nslot) {
                        T fa[SG][KT], fb[SG][KT];
#pragma unroll
                        for (int q = 0; q < SG; ++q) {
                            const int sl = g0 + q < kRdmSlots ? g0 + q : kRdmSlots - 1;
                            if (g0 + q < nslot) {
                                frag(sbi[sl], fa[q]);
                                frag(sbj[sl], fb[q]);
                            }
                        }
#pragma unroll
                        for (int t = 0; t < KT; ++t)
#pragma unroll
                            for (int q = 0; q < SG; ++q)
                                if (g0 + q < kRdmSlots && g0 + q < nslot)
                                    acc[g0 + q] = M::op(fa[q][t], fb[q][t], acc[g0 + q]);
                    }
                    __builtin_amdgcn_sched_barrier(0);         // one group's operands in registers at a time
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < KA; ++i) aval[i] = anext[i];
#pragma unroll
            for (int i = 0; i < KB; ++i) {
                bprev[i] = bw[i];
                bw[i] = bnext[i];
            }
            bs = bsnext;
        }
        // one alpha string's products are summed in the accumulators' precision,
        // the strings of a workgroup in FP64 (each element has one owning lane)
#pragma unroll
        for (int s = 0; s < kRdmSlots; ++s) {
            if (s < nslot) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    double *o = out + int64_t(s0 + s) * 256 + M::out_row(lane, i) * 16 + (lane & 15);
                    *o = (first ? 0.0 : *o) + double(acc[s][i]);
                }
            }
            acc[s] = acc_t{0, 0, 0, 0};
        }
        first = false;
    }
}

// M_tri[pair][256] = sum over workgroups of the partial sums
__global__ __launch_bounds__(256) void k_rdm_reduce(const double *part, int G, int64_t len, double *mtri) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= len) return;
    double s = 0;
    for (int b = 0; b < G; ++b) s += part[int64_t(b) * len + i];
    mtri[i] = s;
}

// element (x, y) of the symmetric M from its upper-triangle blocks
__device__ __forceinline__ double m_at(const double *mtri, int nb, int x, int y) {
    if (x / 16 > y / 16) { const int t = x; x = y; y = t; }
    const int bi = x / 16, bj = y / 16;
    const int pidx = bi * (2 * nb - bi + 1) / 2 + (bj - bi);
    return mtri[int64_t(pidx) * 256 + (x % 16) * 16 + (y % 16)];
}

__global__ __launch_bounds__(256) void k_rdm_final(const double *mtri, int nb, int n, double *rdm1, double *rdm2) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int n2 = n * n;
    const int64_t n4 = int64_t(n2) * n2;
    const double norm = m_at(mtri, nb, n2, n2);
    if (i < n2) rdm1[i] = m_at(mtri, nb, n2, int(i)) / norm;
    if (i >= n4) return;
    const int pq = int(i / n2), rs = int(i % n2);
    const int pp = pq / n, q = pq % n, r = rs / n, s = rs % n;
    double v = m_at(mtri, nb, q * n + pp, rs) / norm;
    if (q == r) v -= m_at(mtri, nb, n2, pp * n + s) / norm;
    rdm2[i] = v;
}

template <typename T>
constexpr int rdm_nt() { return sizeof(T) == 4 ? 32 : 16; }

}  // namespace

int rdm_blocks(int n) { return (n * n + 1 + 15) / 16; }

size_t rdm_lds_bytes(const cisigma_ctx *ctx, int dtype) {
    const int es = dtype == CISIGMA_FP32 ? 4 : 8;
    const int nt = dtype == CISIGMA_FP32 ? rdm_nt<float>() : rdm_nt<double>();
    return size_t(16 * rdm_blocks(ctx->n) * (nt + 16 / es) + ctx->pl[0].ld[0]) * es + size_t(2 * 16 * rdm_blocks(ctx->n)) * 4;
}

int rdm_grid(const cisigma_ctx *ctx) { return std::min(ctx->sp[0].nstr, 256); }

size_t rdm_part_elems(const cisigma_ctx *ctx) {
    const int nb = rdm_blocks(ctx->n);
    const size_t npb = size_t(nb) * (nb + 1) / 2;
    return (size_t(rdm_grid(ctx)) + 1) * npb * 256;   // partials, then the reduced blocks
}

hipError_t launch_rdm(const cisigma_ctx *ctx, const void *cp, int dtype, double *part, double *rdm1, double *rdm2,
                      hipStream_t s) {
    const int nb = rdm_blocks(ctx->n);
    // the kernel holds at most 64 single excitations per string (n <= 16) and 17 row blocks
    if (nb > kRdmMaxBlocks || ctx->sp[0].nexc > 64 || ctx->sp[1].nexc > 64) return hipErrorInvalidValue;
    const int npb = nb * (nb + 1) / 2;
    const int G = rdm_grid(ctx);
    const size_t lds = rdm_lds_bytes(ctx, dtype);
    if (lds > 160 * 1024 || G <= 0) return hipErrorInvalidValue;
    auto fill = [&](auto &a) {
        a.aexc = ctx->sp[0].d_exc;
        a.bexc = ctx->sp[1].d_exc;
        a.astr = ctx->sp[0].d_str;
        a.bstr = ctx->sp[1].d_str;
        a.part = part;
        a.n = ctx->n;
        a.Na = ctx->sp[0].nstr;
        a.Nb = ctx->sp[1].nstr;
        a.ld = ctx->pl[0].ld[0];
        a.anexc = ctx->sp[0].nexc;
        a.bnexc = ctx->sp[1].nexc;
        a.nb = nb;
        a.npb = npb;
    };
    hipError_t e;
    if (dtype == CISIGMA_FP32) {
        RdmArgs<float> a{};
        fill(a);
        a.cp = static_cast<const float *>(cp);
        constexpr int NT = rdm_nt<float>();
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rdm<float, NT>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_rdm<float, NT>), dim3(G), dim3(512), lds, s, a);
    } else {
        RdmArgs<double> a{};
        fill(a);
        a.cp = static_cast<const double *>(cp);
        constexpr int NT = rdm_nt<double>();
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rdm<double, NT>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_rdm<double, NT>), dim3(G), dim3(512), lds, s, a);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t len = int64_t(npb) * 256;
    double *mtri = part + int64_t(G) * len;
    hipLaunchKernelGGL(k_rdm_reduce, dim3(unsigned((len + 255) / 256)), dim3(256), 0, s, part, G, len, mtri);
    const int64_t n4 = int64_t(ctx->n) * ctx->n * ctx->n * ctx->n;
    hipLaunchKernelGGL(k_rdm_final, dim3(unsigned((n4 + 255) / 256)), dim3(256), 0, s, mtri, nb, ctx->n, rdm1, rdm2);
    return hipGetLastError();
}

}  // namespace cis
