// sigma_abg.hip -- owner-computes form of the alpha-beta part sigma_3 (Eq. 8)
// for GAS spaces (Sec. 3.1 occupation types), and for one-block spaces whose
// sigma row is too long for the one-block kernel.  The contraction and the
// beta-side scatter are those of the one-block form (abx.h); what differs is
// which source tiles, k steps and W rows each alpha type needs, and that a
// sigma row holds only the columns of the blocks allowed with the type.
#include "internal.h"
#include "mfma.h"
#include "bufio.h"
#include "abx.h"

#include <algorithm>
#include <type_traits>

namespace cis {
namespace {

// ---- GAS spaces: owner-computes with per-type source tiles ---------------------
//
// Units: an alpha type ta and a range [lo, hi) of its compact columns (the
// beta strings of the blocks allowed with ta, concatenated).  One launch covers
// all units, one workgroup per (unit, alpha string of its type), four waves as
// in the FP64 one-block form.
// The LDS sigma row holds the unit's columns; the unit's plan drops every
// contribution that lands outside them.  For each source tile of the unit (32
// columns of one beta type u2) the gathered rows are the single excitations of
// Ia grouped by source type, each read from its block with u2 (or the zero
// row); only the k steps whose rows have a block with u2 and the W row blocks
// whose pairs lead into a block of ta are multiplied.  W rows of skipped
// blocks are stale and no plan entry reads them.
template <typename T>
struct AbgArgs {
    const T *cp;                 // C, alpha-major padded GAS layout, zero row at zero_off
    T *sp;                       // sigma accumulator, same layout (read, then overwritten)
    const uint32_t *aexc, *astr;
    const int *atype, *astart;   // type of each alpha string, first string of each type
    const int64_t *seg;          // [nta][ntb] block offsets (-1: not in the space)
    const int *ld;               // [ntb] row strides
    const int *bstart;           // [ntb + 1] first beta string of each type
    const T *g;                  // [n*n][mp] (ij|kl), kl in the grouped row order
    const int *slot;             // [nta][4*ks] excitation index of each gathered row (-2: Ia, -1: none)
    const uint4 *act;            // tiles of all units: {plan tile, k-step mask, row-block mask, beta type | first column << 8}
    const int *coff;             // [nta][ntb] first compact column of each allowed block (-1: not allowed)
    const int *units;            // [nunits][8]: ta, lo, hi, act0, nact, first alpha string, first workgroup
    const uint32_t *plan;
    uint32_t cp_bytes, plan_bytes, zero_off;
    int anexc, n, npair, mp, ntb, nunits;
    int nvirt;                   // the longest unit row (LDS layout)
};

template <typename T, int KS, int RB, int EW>
__global__ __launch_bounds__(256, 1) void k_sigma_ab_g(AbgArgs<T> p) {
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    constexpr int RBW = (RB + 1) / 2;
    constexpr int MP = 16 * RB;
    constexpr int KP = 4 * KS;
    constexpr int PW = (EW + 1) * 64;
    constexpr int PT = 4 * PW;
    constexpr int TS = sizeof(T) == 4 ? 2 : 3;              // plan slot fields count elements
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *W = reinterpret_cast<T *>(smem_raw);                // [MP][WS]
    T *sig = W + MP * kAbxWS;                              // [nvirt + 64]
    uint32_t *rowoff = reinterpret_cast<uint32_t *>(sig + p.nvirt + 64);   // [ntb][KP] byte offsets

    int ui = 0;                                            // this workgroup's unit (uniform)
    while (ui + 1 < p.nunits && int(blockIdx.x) >= p.units[8 * (ui + 1) + 6]) ++ui;
    const int *U = p.units + 8 * ui;
    const int ulo = U[1], uhi = U[2], ncol = uhi - ulo;
    const int Ia = U[5] + (int(blockIdx.x) - U[6]);
    const int ta = p.atype[Ia], ra = Ia - p.astart[ta];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cb = wave & 1, grp = wave >> 1;
    const int rb0 = grp == 0 ? 0 : RBW, nrb = grp == 0 ? RBW : RB - RBW;
    const int64_t *segrow = p.seg + int64_t(ta) * p.ntb;
    const int *coff = p.coff + int64_t(ta) * p.ntb;
    // the unit's compact columns [lo, hi): the parts of the allowed blocks of ta inside them
    for (int u = 0; u < p.ntb; ++u) {
        const int o = coff[u];
        if (o < 0) continue;
        const int cnt = p.bstart[u + 1] - p.bstart[u];
        const int x0 = o > ulo ? o : ulo, x1 = o + cnt < uhi ? o + cnt : uhi;
        const T *src = p.sp + segrow[u] + int64_t(ra) * p.ld[u] - o;
        for (int x = x0 + tid; x < x1; x += 256) sig[x - ulo] = src[x];
    }
    const int *sl = p.slot + int64_t(ta) * KP;
    for (int idx = tid; idx < KP * p.ntb; idx += 256) {
        const int u = idx / KP, q = idx % KP;
        const int e = sl[q];
        int Ja = -1;
        if (e == -2) {
            Ja = Ia;
        } else if (e >= 0) {
            const uint32_t w = p.aexc[int64_t(Ia) * p.anexc + e];
            if (w != kExcNone) Ja = int(w >> 11);
        }
        uint32_t off = p.zero_off;
        if (Ja >= 0) {
            const int t2 = p.atype[Ja];
            const int64_t s = p.seg[int64_t(t2) * p.ntb + u];
            if (s >= 0) off = uint32_t(s + int64_t(Ja - p.astart[t2]) * p.ld[u]);
        }
        rowoff[idx] = off * uint32_t(sizeof(T));
    }
    // A fragments: row m (grouped pair order) = 16*(rb0 + r) + lane%16, gathered row 4t + lane/16
    T A[RBW][KS];
    const uint32_t xa = p.astr[Ia];
#pragma unroll
    for (int t = 0; t < KS; ++t) {
        const int e = sl[4 * t + (lane >> 4)];
        const T *g = nullptr;
        T sg = 0;
        if (e >= 0) {
            const uint32_t w = p.aexc[int64_t(Ia) * p.anexc + e];
            if (w != kExcNone) {
                const int i = (w >> 6) & 31, j = (w >> 1) & 31;   // <Ia|E_ij|Ja>, Ja = Ia - i + j
                g = p.g + int64_t(i * p.n + j) * p.mp;
                sg = (w & 1) ? T(-1) : T(1);
            }
        }
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
            const int m = (rb0 + r) * 16 + (lane & 15);
            T val = 0;
            if (r < nrb && m < p.npair) {
                if (g) {
                    val = sg * g[m];
                } else if (e == -2) {
                    for (uint32_t b = xa; b; b &= b - 1) {
                        const int j = __ffs(b) - 1;
                        val += p.g[int64_t(j * p.n + j) * p.mp + m];
                    }
                }
            }
            A[r][t] = val;
        }
    }
    __syncthreads();

    const int nact = U[4];
    if (nact > 0) {
        const __amdgpu_buffer_rsrc_t cr = buffer_of(p.cp, p.cp_bytes), pr = buffer_of(p.plan, p.plan_bytes);
        const uint32_t colb = uint32_t(cb * 16 + (lane & 15)) * uint32_t(sizeof(T));
        const uint32_t pl = uint32_t(wave * PW + lane) * 4u;
        const uint32_t spare = uint32_t(ncol + lane) * uint32_t(sizeof(T));
        const uint4 *act = p.act + U[3];
        T bc[KS], bn[KS];
        acc_t acc[RBW], acc2[RBW];
        // gathered rows of an item for every k step: one LDS offset read each
        // (only the k steps the item multiplies: the others read the zero row anyway)
        auto load = [&](const uint4 &e, T (&b)[KS]) {
            const uint32_t *ro = rowoff + (e.w & 255u) * KP + (lane >> 4);
            const uint32_t soff = (e.w >> 8) * uint32_t(sizeof(T));
#pragma unroll
            for (int t = 0; t < KS; ++t) {
                if ((e.y >> t) & 1u) buffer_ld(b[t], cr, ro[4 * t] + colb, soff);
                else b[t] = T(0);
            }
        };
        // two accumulators per row block (even and odd k steps): independent MFMA
        // chains.  FP64: only the item's active k steps (a uniform branch each);
        // FP32: the k steps in four chunks, a chunk multiplied when one of its k
        // steps is active (measured at GAS(20,20): FP64 148 ms per-step vs 159 ms
        // chunked, FP32 79 ms chunked vs 88 ms per-step)
        constexpr bool PER_STEP = sizeof(T) == 8;
        constexpr uint32_t CM0 = PER_STEP ? 1u : (1u << (KS / 4)) - 1u;
        constexpr uint32_t CM1 = ((1u << (KS / 2)) - 1u) & ~CM0;
        constexpr uint32_t CM2 = ((1u << (3 * KS / 4)) - 1u) & ~(CM0 | CM1);
        constexpr uint32_t CM3 = (KS == 32 ? 0xffffffffu : ((1u << KS) - 1u)) & ~(CM0 | CM1 | CM2);
        auto products = [&](uint32_t km, uint32_t rm) {
#pragma unroll
            for (int r = 0; r < RBW; ++r) {
                acc[r] = acc_t{0, 0, 0, 0};
                acc2[r] = acc_t{0, 0, 0, 0};
                if (r >= nrb || !((rm >> (rb0 + r)) & 1u)) continue;
                if (PER_STEP) {
#pragma unroll
                    for (int t = 0; t < KS; ++t) {
                        if (!((km >> t) & 1u)) continue;
                        if (t & 1) acc2[r] = M::op(A[r][t], bc[t], acc2[r]);
                        else acc[r] = M::op(A[r][t], bc[t], acc[r]);
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const uint32_t cm = c == 0 ? CM0 : c == 1 ? CM1 : c == 2 ? CM2 : CM3;
                        if (!(km & cm)) continue;
#pragma unroll
                        for (int t = 0; t < KS; ++t) {
                            if (!((cm >> t) & 1u)) continue;
                            if (t & 1) acc2[r] = M::op(A[r][t], bc[t], acc2[r]);
                            else acc[r] = M::op(A[r][t], bc[t], acc[r]);
                        }
                    }
                }
                acc[r] += acc2[r];
            }
        };
        auto store_w = [&](uint32_t rm) {
#pragma unroll
            for (int r = 0; r < RBW; ++r)
                if (r < nrb && ((rm >> (rb0 + r)) & 1u))
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        W[((rb0 + r) * 16 + M::out_row(lane, i)) * kAbxWS + cb * 16 + (lane & 15)] = acc[r][i];
        };
        // items i + 1 and i + 2 are read one iteration ahead of their use
        uint4 e1 = act[nact > 1 ? 1 : 0], e2 = act[nact > 2 ? 2 : nact - 1];
        {
            const uint4 e0 = act[0];
            load(e0, bc);
            load(e1, bn);
            products(e0.y, e0.z);
            store_w(e0.z);
        }
        // act .x: plan tile | its entries per lane << 24
        uint32_t pw_[EW], ph, nw_[EW], nh;
        int pn = int(act[0].x >> 24), nn = 0;
        abx_plan_load_n<EW>(pr, pl, (act[0].x & 0xffffffu) * (PT * 4u), pw_, ph, pn);
        __syncthreads();
        for (int i = 0; i < nact; ++i) {
            const bool more = i + 1 < nact;
            const uint4 e3 = act[i + 3 < nact ? i + 3 : nact - 1];
#pragma unroll
            for (int t = 0; t < KS; ++t) bc[t] = bn[t];          // rows of item i + 1
            load(e2, bn);                                        // item i + 2, in flight for a whole item
            nn = int(e1.x >> 24);
            abx_plan_load_n<EW>(pr, pl, (e1.x & 0xffffffu) * (PT * 4u), nw_, nh, nn);
            products(more ? e1.y : 0u, e1.z);                    // next item's W (after the last: nothing)
            abx_scatter_n<T, EW, TS>(W, sig, pw_, ph, spare, pn);
            __syncthreads();                                     // W of this item consumed
            if (more) store_w(e1.z);
            __syncthreads();
#pragma unroll
            for (int q = 0; q < EW; ++q) pw_[q] = nw_[q];
            ph = nh;
            pn = nn;
            e1 = e2;
            e2 = e3;
        }
    }
    for (int u = 0; u < p.ntb; ++u) {
        const int o = coff[u];
        if (o < 0) continue;
        const int cnt = p.bstart[u + 1] - p.bstart[u];
        const int x0 = o > ulo ? o : ulo, x1 = o + cnt < uhi ? o + cnt : uhi;
        T *dst = p.sp + segrow[u] + int64_t(ra) * p.ld[u] - o;
        for (int x = x0 + tid; x < x1; x += 256) dst[x] = sig[x - ulo];
    }
}

template <typename T>
size_t abg_lds(int nvirt, int rb, int ks, int ntb) {
    return (size_t(16) * rb * kAbxWS + nvirt + 64) * sizeof(T) + size_t(4) * ks * ntb * sizeof(uint32_t);
}

template <typename T, int KS, int RB, int EW>
hipError_t run_abg(const AbgArgs<T> &a, int na, hipStream_t s) {
    const size_t lds = abg_lds<T>(a.nvirt, RB, KS, a.ntb);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sigma_ab_g<T, KS, RB, EW>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sigma_ab_g<T, KS, RB, EW>), dim3(na), dim3(256), lds, s, a);
    return hipGetLastError();
}

// compiled (KS, RB, EW) shapes of the GAS kernel: small test spaces, GAS(20,20)
// 6/8/6 and CAS(18,18) (whose sigma row is too long for the one-block kernel)
#define CIS_ABG_SHAPES(X) \
    X(3, 2, 4) X(3, 2, 16) X(4, 2, 4) X(4, 2, 16) X(4, 3, 4) X(4, 3, 16) X(26, 14, 16) \
    X(21, 11, 8) X(21, 11, 12) X(21, 11, 16)

int gas_width_for(int ks, int rb, int need) {
    int best = 0;
#define CIS_W(K, R, E) if (ks == K && rb == R && E >= need && (best == 0 || E < best)) best = E;
    CIS_ABG_SHAPES(CIS_W)
#undef CIS_W
    return best;
}

template <typename T>
bool gas_t(const cisigma_ctx *ctx, const void *cp, void *sp, hipStream_t s, hipError_t *err) {
    const GasOwner &G = ctx->go;
    const int d = sizeof(T) == 4 ? 1 : 0;
    const uint32_t *plan = G.plan[d].d_entries[d];
    if (G.ks == 0 || !plan || G.plan[d].ew == 0 || G.units[d].empty()) return false;
    const auto &A = ctx->sp[0];
    const auto &L = ctx->pl[0];
    int64_t ldmax = 0;
    for (int v : L.ld) ldmax = std::max<int64_t>(ldmax, v);
    const uint64_t cpb = (uint64_t(L.size) + uint64_t(ldmax)) * sizeof(T);
    const uint64_t plb = uint64_t(G.plan[d].ntile) * 4 * (G.plan[d].ew + 1) * 64 * sizeof(uint32_t);
    if (cpb >= (uint64_t(1) << 31) || plb >= (uint64_t(1) << 31)) return false;
    bool shape = false;
#define CIS_HAS(K, R, E) shape = shape || (G.ks == K && G.rb == R && G.plan[d].ew == E);
    CIS_ABG_SHAPES(CIS_HAS)
#undef CIS_HAS
    if (!shape) return false;
    AbgArgs<T> a{};
    a.cp = static_cast<const T *>(cp);
    a.sp = static_cast<T *>(sp);
    a.aexc = A.d_exc;
    a.astr = A.d_str;
    a.atype = A.d_stype;
    a.astart = ctx->d_tstart[0];
    a.seg = L.d_seg;
    a.ld = L.d_ld;
    a.bstart = ctx->d_tstart[1];
    a.g = std::is_same<T, float>::value ? reinterpret_cast<const T *>(G.d_g32) : reinterpret_cast<const T *>(G.d_g64);
    a.slot = G.d_slot;
    a.coff = G.d_coff;
    a.plan = plan;
    a.cp_bytes = uint32_t(cpb);
    a.plan_bytes = uint32_t(plb);
    a.zero_off = uint32_t(L.size);
    a.anexc = A.nexc;
    a.n = ctx->n;
    a.npair = ctx->npair;
    a.mp = 16 * G.rb;
    a.ntb = ctx->sp[1].ntype;
    a.act = reinterpret_cast<const uint4 *>(G.d_act[d]);
    a.units = G.d_units[d];
    a.nunits = int(G.units[d].size());
    a.nvirt = G.maxcols[d];
    int *kshape = const_cast<cisigma_ctx *>(ctx)->last_shape[sizeof(T) == 4];
#define CIS_RUN(K, R, E)                                                \
    if (G.ks == K && G.rb == R && G.plan[d].ew == E) {                  \
        *err = run_abg<T, K, R, E>(a, G.nblocks[d], s);                 \
        kshape[0] = K; kshape[1] = R; kshape[2] = E; kshape[3] = 3;     \
    }
    CIS_ABG_SHAPES(CIS_RUN)
#undef CIS_RUN
    return true;
}

}  // namespace

int sigma_ab_gas_width(int ks, int rb, int need) { return gas_width_for(ks, rb, need); }

bool launch_sigma_ab_gas(const cisigma_ctx *ctx, const void *cp, void *sp, int dtype, hipStream_t s,
                         hipError_t *err) {
    return dtype == CISIGMA_FP32 ? gas_t<float>(ctx, cp, sp, s, err) : gas_t<double>(ctx, cp, sp, s, err);
}

}  // namespace cis
