// sigma_ab.hip -- the alpha-beta part sigma_3 of the sigma vector (Eq. 8):
//
//   sigma_3(Ia, Ib) = sum_{ij,kl} (ij|kl) sum_Ja <Ia|E^a_ij|Ja> sum_Jb <Ib|E^b_kl|Jb> C(Ja, Jb)
//
// string-driven (Sec. 3.3) and organised around one dense contraction per
// source alpha string Ja (the "loops over types of excitations, each a matrix
// multiply" of Sec. 4):
//
//   D(kl, Ib)  = sum_Jb <Ib|E^b_kl + E^b_lk|Jb> C(Ja, Jb)     gathered from the C row of Ja
//                (kl = unordered pair k >= l; the diagonal kk rows are C(Ja, Ib) n_k(Ib))
//   F(a, Ib)   = sum_kl s_a (i_a j_a|kl) D(kl, Ib)             MFMA, a = alpha excitations of Ja
//   sigma(Ia_a, Ib) += F(a, Ib)                                 scatter (hardware float atomics)
//
// with a running over the off-diagonal alpha excitations Ia_a = a^+_i a_j Ja
// (sign s_a).  The alpha-diagonal terms (i = j in Ja, Ia = Ja) contribute
// sum_kl v(kl) D(kl, Ib), v(kl) = sum_{j in Ja} (jj|kl); they are summed on the
// vector ALU while D is gathered.
#include "internal.h"
#include "mfma.h"

#include <algorithm>
#include <type_traits>

namespace cis {
namespace {


template <typename T>
struct AbArgs {
    const T *cp;                 // C, alpha-major padded layout
    T *sp;                       // sigma accumulator, alpha-major padded layout
    const uint32_t *aexc;        // [Na][anexc]
    const uint32_t *bexc;        // [Nb][bnexc]
    const uint32_t *bstr;        // [Nb]
    const uint32_t *astr;        // [Na]
    const int *atype, *btype;    // type of each string
    const int *astart, *bstart;  // first string of each type
    const int64_t *seg;          // [nta][ntb]
    const int *ld;               // [ntb]
    const int *tile_u, *tile_c0; // 64-column tiles of the beta types
    const int *act_start, *act_tiles;   // per alpha type: the tiles that can change sigma
    const T *gp;                 // [n*n][kp]
    int anexc, bnexc, ntb, ntiles;
    int n, kp, Na, Nb;
    int stage;                   // C row of Ja staged in LDS
    int act_max;                 // longest active-tile list
};

__device__ __forceinline__ float neg_if(float v, uint32_t s) { return s ? -v : v; }
__device__ __forceinline__ double neg_if(double v, uint32_t s) { return s ? -v : v; }

// KS: 4-wide k steps (kp = 4 KS); RBW: 16-row blocks per wave; NT: tile columns
template <typename T, int KS, int RBW, int NT>
__global__ __launch_bounds__(256) void k_sigma_ab(AbArgs<T> p) {
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    constexpr int KP = 4 * KS;
    constexpr int DS = NT + (sizeof(T) == 4 ? 16 : 0);   // LDS row stride of D (bank spread)
    constexpr int TPC = 256 / NT;                         // threads per D column
    constexpr int NCB = NT / 16;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *v = reinterpret_cast<T *>(smem_raw);
    T *D = v + KP;
    T *crow = D + KP * DS;

    const int Ja = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ta = p.atype[Ja];
    const int ra = Ja - p.astart[ta];
    const int64_t *segrow = p.seg + int64_t(ta) * p.ntb;

    // stage the C row of Ja as a virtual row over all beta strings
    if (p.stage) {
        for (int u = 0; u < p.ntb; ++u) {
            int b0 = p.bstart[u], cnt = p.bstart[u + 1] - b0;
            int64_t s = segrow[u];
            if (s >= 0) {
                const T *src = p.cp + s + int64_t(ra) * p.ld[u];
                for (int i = tid; i < cnt; i += 256) crow[b0 + i] = src[i];
            } else {
                for (int i = tid; i < cnt; i += 256) crow[b0 + i] = T(0);
            }
        }
    }
    // v(kl) = sum_{j in Ja} (jj|kl)
    const uint32_t xa = p.astr[Ja];
    for (int q = tid; q < KP; q += 256) {
        T s = 0;
        for (uint32_t b = xa; b; b &= b - 1) {
            int j = __ffs(b) - 1;
            s += p.gp[int64_t(j * p.n + j) * KP + q];
        }
        v[q] = s;
    }
    // A fragments: row a = 16*rb + lane%16, k = 4t + lane/16; sign folded in
    T A[RBW][KS];
    int tgt[RBW][4];
#pragma unroll
    for (int r = 0; r < RBW; ++r) {
        const int rb = wave + 4 * r;
        const int a = rb * 16 + (lane & 15);
        uint32_t e = (a < p.anexc) ? p.aexc[int64_t(Ja) * p.anexc + a] : kExcNone;
        const T *g = nullptr;
        T sg = 0;
        if (e != kExcNone) {
            int kk = (e >> 6) & 31, ll = (e >> 1) & 31;   // Ia = a^+_ll a_kk Ja
            g = p.gp + int64_t(ll * p.n + kk) * KP;
            sg = (e & 1) ? T(-1) : T(1);
        }
#pragma unroll
        for (int t = 0; t < KS; ++t) A[r][t] = g ? sg * g[4 * t + (lane >> 4)] : T(0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ao = rb * 16 + M::out_row(lane, i);
            uint32_t eo = (ao < p.anexc) ? p.aexc[int64_t(Ja) * p.anexc + ao] : kExcNone;
            tgt[r][i] = (eo == kExcNone) ? -1 : int(eo >> 11);
        }
    }
    __syncthreads();

    const T *crow_g_base = nullptr;   // direct row pointer when not staged and single beta type
    if (!p.stage && p.ntb == 1 && segrow[0] >= 0) crow_g_base = p.cp + segrow[0] + int64_t(ra) * p.ld[0];

    constexpr int HALVES = kTileCols / NT;   // a 64-column layout tile in NT-column pieces
    const int act0 = p.act_start[ta], nact = p.act_start[ta + 1] - act0;
    for (int item = blockIdx.y; item < nact * HALVES; item += gridDim.y) {
        const int tile = p.act_tiles[act0 + item / HALVES];
        const int u = p.tile_u[tile], c0 = p.tile_c0[tile] + (item % HALVES) * NT;
        const int b0 = p.bstart[u], cnt = p.bstart[u + 1] - b0;
        for (int i = tid; i < KP * DS; i += 256) D[i] = T(0);
        __syncthreads();
        // ---- gather D(kl, Ib) for the tile's output beta strings
        const int c = tid / TPC, sub = tid % TPC;
        const int cc = c0 + c;
        T dsum = 0;
        if (cc < cnt) {
            const int Ib = b0 + cc;
            auto loadc = [&](int Jb) -> T {
                if (p.stage) return crow[Jb];
                if (crow_g_base) return crow_g_base[Jb];
                int uj = p.btype[Jb];
                int64_t s = segrow[uj];
                return s < 0 ? T(0) : p.cp[s + int64_t(ra) * p.ld[uj] + (Jb - p.bstart[uj])];
            };
            const uint32_t *L = p.bexc + int64_t(Ib) * p.bnexc;
            for (int e = sub; e < p.bnexc; e += TPC) {
                uint32_t w = L[e];
                if (w == kExcNone) continue;
                int Jb = int(w >> 11), k = (w >> 6) & 31, l = (w >> 1) & 31;
                T val = neg_if(loadc(Jb), w & 1);
                int q = pair_ge(k, l);
                D[q * DS + c] = val;
                dsum += v[q] * val;
            }
            const T cv = loadc(Ib);
            int cntb = 0;
            for (uint32_t b = p.bstr[Ib]; b; b &= b - 1, ++cntb) {
                if (cntb % TPC != sub) continue;
                int k = __ffs(b) - 1;
                int q = k * (k + 1) / 2 + k;
                D[q * DS + c] = cv;
                dsum += v[q] * cv;
            }
        }
#pragma unroll
        for (int off = TPC / 2; off > 0; off >>= 1) dsum += __shfl_xor(dsum, off);
        if (sub == 0 && cc < cnt) {
            int64_t s = segrow[u];
            if (s >= 0) unsafeAtomicAdd(p.sp + s + int64_t(ra) * p.ld[u] + cc, dsum);
        }
        __syncthreads();
        // ---- F = A D on the matrix cores
        acc_t acc[RBW][NCB];
#pragma unroll
        for (int r = 0; r < RBW; ++r)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[r][cb] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < KS; ++t) {
            const T *drow = D + (4 * t + (lane >> 4)) * DS + (lane & 15);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                T b = drow[cb * 16];
#pragma unroll
                for (int r = 0; r < RBW; ++r) acc[r][cb] = M::op(A[r][t], b, acc[r][cb]);
            }
        }
        // ---- scatter F into the sigma rows Ia_a
#pragma unroll
        for (int r = 0; r < RBW; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int Ia = tgt[r][i];
                if (Ia < 0) continue;
                int t2 = p.atype[Ia];
                int64_t s = p.seg[int64_t(t2) * p.ntb + u];
                if (s < 0) continue;
                T *dst = p.sp + s + int64_t(Ia - p.astart[t2]) * p.ld[u] + c0 + (lane & 15);
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
                    if (c0 + cb * 16 + (lane & 15) < cnt) unsafeAtomicAdd(dst + cb * 16, acc[r][cb][i]);
            }
        __syncthreads();
    }
}

// Direct (non-matrix-core) form of sigma_3, one thread per output element;
// used when the orbital count exceeds what the tiled kernel is built for.
template <typename T>
__global__ __launch_bounds__(256) void k_sigma_ab_direct(AbArgs<T> p, int64_t total_rows_cols) {
    int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (id >= total_rows_cols) return;
    const int Ia = int(id / p.Nb), Ib = int(id % p.Nb);
    const int ta = p.atype[Ia], tb = p.btype[Ib];
    const int64_t so = p.seg[int64_t(ta) * p.ntb + tb];
    if (so < 0) return;
    const int KP = p.kp, n = p.n;
    const uint32_t xa = p.astr[Ia], xb = p.bstr[Ib];
    const int na = __popc(xa), nb = __popc(xb);
    T acc = 0;
    // alpha terms: off-diagonal entries of Ia's list plus the diagonal E_pp, p in Ia
    for (int ea = 0; ea < p.anexc + na; ++ea) {
        int Ja, ia, ja;
        T sa;
        if (ea < p.anexc) {
            uint32_t w = p.aexc[int64_t(Ia) * p.anexc + ea];
            if (w == kExcNone) continue;
            Ja = int(w >> 11); ia = (w >> 6) & 31; ja = (w >> 1) & 31; sa = (w & 1) ? T(-1) : T(1);
        } else {
            uint32_t b = xa;
            for (int s = 0; s < ea - p.anexc; ++s) b &= b - 1;
            Ja = Ia; ia = ja = __ffs(b) - 1; sa = 1;
        }
        const int tja = p.atype[Ja];
        const int rja = Ja - p.astart[tja];
        const T *g = p.gp + int64_t(ia * n + ja) * KP;
        for (int eb = 0; eb < p.bnexc + nb; ++eb) {
            int Jb, kb, lb;
            T sb;
            if (eb < p.bnexc) {
                uint32_t w = p.bexc[int64_t(Ib) * p.bnexc + eb];
                if (w == kExcNone) continue;
                Jb = int(w >> 11); kb = (w >> 6) & 31; lb = (w >> 1) & 31; sb = (w & 1) ? T(-1) : T(1);
            } else {
                uint32_t b = xb;
                for (int s = 0; s < eb - p.bnexc; ++s) b &= b - 1;
                Jb = Ib; kb = lb = __ffs(b) - 1; sb = 1;
            }
            const int tjb = p.btype[Jb];
            const int64_t s = p.seg[int64_t(tja) * p.ntb + tjb];
            if (s < 0) continue;
            acc += sa * sb * g[pair_ge(kb, lb)] * p.cp[s + int64_t(rja) * p.ld[tjb] + (Jb - p.bstart[tjb])];
        }
    }
    unsafeAtomicAdd(p.sp + so + int64_t(Ia - p.astart[ta]) * p.ld[tb] + (Ib - p.bstart[tb]), acc);
}

template <typename T, int KS, int RBW, int NT>
hipError_t run_ab(const AbArgs<T> &a, hipStream_t s) {
    constexpr int KP = 4 * KS;
    constexpr int DS = NT + (sizeof(T) == 4 ? 16 : 0);
    size_t lds = size_t(KP + KP * DS) * sizeof(T);
    AbArgs<T> p = a;
    const size_t lds_max = 160 * 1024;
    size_t lds_stage = lds + size_t(a.Nb) * sizeof(T);
    p.stage = lds_stage <= lds_max ? 1 : 0;
    size_t lds_use = p.stage ? lds_stage : lds;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sigma_ab<T, KS, RBW, NT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_use));
    if (e != hipSuccess) return e;
    // enough workgroups to fill the chip when there are few alpha strings
    const int items = std::max(a.act_max, 1) * (kTileCols / NT);
    int ysplit = 1;
    while (int64_t(a.Na) * ysplit < 2048 && ysplit < items) ysplit *= 2;
    if (ysplit > items) ysplit = items;
    hipLaunchKernelGGL((k_sigma_ab<T, KS, RBW, NT>), dim3(a.Na, ysplit), dim3(256), lds_use, s, p);
    return hipGetLastError();
}

template <typename T, int RBW>
hipError_t dispatch_ks(const AbArgs<T> &a, hipStream_t s, int ks) {
    constexpr int NT = sizeof(T) == 4 ? 64 : 32;
    switch (ks) {
#define CIS_KS(K) case K: return run_ab<T, K, RBW, NT>(a, s);
        CIS_KS(2) CIS_KS(4) CIS_KS(6) CIS_KS(8) CIS_KS(10) CIS_KS(12) CIS_KS(14) CIS_KS(18) CIS_KS(20)
        CIS_KS(24) CIS_KS(28) CIS_KS(30) CIS_KS(34) CIS_KS(40) CIS_KS(44) CIS_KS(48) CIS_KS(54) CIS_KS(58)
        CIS_KS(64)
#undef CIS_KS
        default: return hipErrorInvalidValue;
    }
}

// k-step count actually compiled for a given kp: round up to the next instantiated value
int ks_for(int kp) {
    static const int vals[] = {2, 4, 6, 8, 10, 12, 14, 18, 20, 24, 28, 30, 34, 40, 44, 48, 54, 58, 64};
    int need = (kp + 3) / 4;
    for (int v : vals)
        if (v >= need) return v;
    return -1;
}

template <typename T>
hipError_t sigma_ab_t(const cisigma_ctx *ctx, const void *cp, void *sp, hipStream_t s) {
    const auto &A = ctx->sp[0];
    const auto &B = ctx->sp[1];
    const auto &L = ctx->pl[0];
    AbArgs<T> a{};
    a.cp = static_cast<const T *>(cp);
    a.sp = static_cast<T *>(sp);
    a.aexc = A.d_exc;
    a.bexc = B.d_exc;
    a.astr = A.d_str;
    a.bstr = B.d_str;
    a.atype = A.d_stype;
    a.btype = B.d_stype;
    a.astart = ctx->d_tstart[0];
    a.bstart = ctx->d_tstart[1];
    a.seg = L.d_seg;
    a.ld = L.d_ld;
    a.tile_u = L.d_tile_u;
    a.tile_c0 = L.d_tile_c0;
    a.act_start = ctx->d_act_start;
    a.act_tiles = ctx->d_act_tiles;
    a.act_max = ctx->act_max;
    a.anexc = A.nexc;
    a.bnexc = B.nexc;
    a.ntb = B.ntype;
    a.ntiles = L.ntiles;
    a.n = ctx->n;
    a.Na = A.nstr;
    a.Nb = B.nstr;
    a.stage = 0;
    a.gp = std::is_same<T, float>::value ? reinterpret_cast<const T *>(ctx->d_gp32)
                                         : reinterpret_cast<const T *>(ctx->d_gp64);
    int ks = ks_for(ctx->kp);
    a.kp = ctx->kp;
    if (ctx->ab_mode != 1) {
        hipError_t e = hipSuccess;
        const int dt = sizeof(T) == 4 ? CISIGMA_FP32 : CISIGMA_FP64;
        // one-block spaces: the one-block owner kernel when its sigma row fits (unless
        // path 2 asks for the units), else the GAS owner kernel (which splits long rows
        // over units), else the general kernel
        const bool one = ctx->cas && ctx->ab_mode != 2 && launch_sigma_ab_owner(ctx, cp, sp, dt, s, &e);
        if (one || launch_sigma_ab_gas(ctx, cp, sp, dt, s, &e)) {
            if (e == hipSuccess) {
                int &f = const_cast<cisigma_ctx *>(ctx)->last_path[sizeof(T) == 4];
                f |= CISIGMA_PATH_AB_OWNER;
                if (one && ctx->abx_shared[sizeof(T) == 4]) f |= CISIGMA_PATH_AB_SHARED_CU;
            }
            return e;
        }
    }
    // the general kernel accumulates with float atomics: refused in deterministic mode
    if (ctx->deterministic) return hipErrorNotSupported;
    const int mb = (A.nexc + 15) / 16;   // 16-row blocks of alpha excitations
    if (ks > 0 && ks * 4 == ctx->kp && mb <= 8) {
        if (mb <= 4) return dispatch_ks<T, 1>(a, s, ks);
        return dispatch_ks<T, 2>(a, s, ks);
    }
    int64_t tot = int64_t(a.Na) * a.Nb;
    hipLaunchKernelGGL((k_sigma_ab_direct<T>), dim3(unsigned((tot + 255) / 256)), dim3(256), 0, s, a, tot);
    return hipGetLastError();
}

}  // namespace

// kp (the padded K extent of the integral table) must equal 4*ks_for(npair)
int sigma_ab_kp(int npair) {
    int ks = ks_for(npair);
    return ks > 0 ? 4 * ks : ((npair + 3) / 4) * 4;
}

hipError_t launch_sigma_ab(const cisigma_ctx *ctx, const void *cp, void *sp, int dtype, hipStream_t s) {
    if (ctx->na == 0 || ctx->nb == 0) return hipSuccess;
    return dtype == CISIGMA_FP32 ? sigma_ab_t<float>(ctx, cp, sp, s) : sigma_ab_t<double>(ctx, cp, sp, s);
}

}  // namespace cis
