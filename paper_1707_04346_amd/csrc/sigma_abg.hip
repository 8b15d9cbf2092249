// sigma_abg.hip -- owner-computes form of the alpha-beta part sigma_3 (Eq. 8)
// for spaces with several string types (GAS occupation types and point-group
// irreps, Sec. 3.1), and for one-block spaces whose sigma row is too long for
// the one-block kernel.  The contraction and the
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

// Unit and item tables are the same for every lane: reading them through
// readfirstlane keeps the values in scalar registers, so plan loads take them as
// scalar offsets and the row-block and k-step masks become scalar branches
// (read as per-lane values they turned every plan load into a loop over lanes
// and every masked MFMA into a masked one)
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uni(uint32_t v) { return uint32_t(__builtin_amdgcn_readfirstlane(int(v))); }
__device__ __forceinline__ uint4 uni_ld(const uint4 *p) {
    const uint4 v = *p;
    return make_uint4(uni(v.x), uni(v.y), uni(v.z), uni(v.w));
}

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
    uint32_t plan_bytes, zero_off;   // zero_off: element index of the zero row (C may exceed 4 GB)
    uint32_t cp_bytes;               // bytes of C with its zero row when below 4 GB, else 0
    int ld0;                         // row stride of one-block spaces (the eight-wave unit kernel)
    int block_base;                  // workgroup index of blockIdx 0 (one launch per unit: its first)
    int anexc, n, mp, ntb, nunits;   // mp: W rows (pair rows with gaps; unused rows have zero integrals)
    int nvirt;                   // the longest unit row (LDS layout)
    int rtk;                     // 1 (point-group spaces): LDS for the per-beta-type k-step masks
};

// abx_scatter_n over the entries in chunks of CH: the W values and old sigma
// values of one chunk in registers at a time (a lane writes each real target
// once, at the end of its group, so a later chunk never reads a slot an earlier
// one wrote except the lane's discard slot).  With all 16 entries' operands
// loaded first the eight-wave FP32 form spilled 132 bytes per lane; in chunks of
// 4, none: GAS(20,20) sigma_3 FP32 57.6 -> 52.6 ms, FP64 115.6 -> 93.8 ms (its
// spill 552 -> 244 bytes)
template <typename T, int EW, int TS, int CH>
__device__ __forceinline__ void abg_scatter_ch(const T *W, T *sig, const uint32_t (&w)[EW], uint32_t hdr,
                                               uint32_t spare, int n) {
    const char *wb = reinterpret_cast<const char *>(W);
    char *sb = reinterpret_cast<char *>(sig);
    T run = 0;
    bool any_start = (hdr & 1u) != 0;
    uint32_t last = spare;
#pragma unroll
    for (int c0 = 0; c0 < EW; c0 += CH) {
        if (c0 >= n) break;
        T val[CH], old[CH];
        uint32_t t[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            if (c0 + q >= n) break;
            t[q] = (w[c0 + q] >> 16) << TS;
            val[q] = flip_if(*reinterpret_cast<const T *>(wb + (w[c0 + q] & 0xfffeu)), w[c0 + q]);
            old[q] = *reinterpret_cast<const T *>(sb + t[q]);
        }
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            if (c0 + q >= n) break;
            const bool st = c0 + q == 0 ? (hdr & 1u) != 0 : last != spare;
            any_start = any_start || st;
            run = st ? val[q] : run + val[q];
            *reinterpret_cast<T *>(sb + t[q]) = old[q] + run;
            last = t[q];
        }
    }
    const T tail = last != spare ? T(0) : run;
    const T carry = carry3<T>(tail, any_start ? 1 : 0);
    T *d = reinterpret_cast<T *>(sb + (hdr & ~3u));
    *d = *d + carry;
}

template <typename T, int KS, int RB, int EW, int NW, bool RTK>
__global__ __launch_bounds__(64 * NW, 1) void k_sigma_ab_g(AbgArgs<T> p) {
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    constexpr int NT = 64 * NW;                             // threads
    // FP64 shapes whose half of the A fragments alone would take more than 320
    // registers per lane: every wave multiplies both 16-column halves for a quarter
    // of the row blocks (strided over the waves), so it holds a quarter of the
    // fragments (GAS(20,20), 26 k steps x 14 row blocks: 234 registers spilled
    // before; sigma_3 93.7 -> 82.9 ms).  Smaller shapes keep two row groups x two
    // column halves: the strided split leaves their row blocks uneven (CAS(16,16)
    // D2h, 9 row blocks: 84.1 -> 92.6 ms with it).
    constexpr bool FC = sizeof(T) == 8 && (RB + 1) / 2 * KS * 2 > 320;
    constexpr int NH = FC ? 2 : 1;                          // column halves per wave
    constexpr int NG = FC ? NW : NW / 2;                    // row-block groups (x 2 / NH column halves)
    // eight waves: gathers as 32-bit byte offsets through a buffer resource (C
    // below 4 GB), one address register per load instead of two
    constexpr bool BUF = NW == 8;
    constexpr int RBW = (RB + NG - 1) / NG;
    constexpr int MP = 16 * RB;
    constexpr int KP = 4 * KS;
    constexpr int PW = (EW + 1) * 64;
    constexpr int PT = 4 * PW;
    constexpr int TS = sizeof(T) == 4 ? 2 : 3;              // plan slot fields count elements
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *W = reinterpret_cast<T *>(smem_raw);                // [MP][WS]
    T *sig = W + MP * kAbxWS;                              // [nvirt + 64]
    uint32_t *rowoff = reinterpret_cast<uint32_t *>(sig + p.nvirt + 64);   // [ntb][KP] element offsets

    const int vb = int(blockIdx.x) + p.block_base;         // this workgroup in the unit table
    int ui = 0;                                            // this workgroup's unit (uniform)
    while (ui + 1 < p.nunits && vb >= uni(p.units[8 * (ui + 1) + 6])) ++ui;
    const int *U = p.units + 8 * uni(ui);
    const int ulo = uni(U[1]), uhi = uni(U[2]), ncol = uhi - ulo;
    const int Ia = uni(U[5]) + (vb - uni(U[6]));
    const int ta = p.atype[Ia], ra = Ia - p.astart[ta];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: the scatter role branches per wave
    const int cb = FC ? 0 : wave & 1, grp = FC ? wave : wave >> 1;
    const int rb0 = FC ? grp : grp * RBW;
    const int nrb = FC ? (RB - grp + NG - 1) / NG : RB - rb0 < RBW ? RB - rb0 : RBW;   // nrb may be <= 0
    // row block of the wave's r-th fragment row: a contiguous run, or every NG-th (FC)
    auto rbi = [&](int r) { return FC ? rb0 + NG * r : rb0 + r; };
    const bool scat = wave < 4;                            // the tile plan's four wave ranges
    const int64_t *segrow = p.seg + int64_t(ta) * p.ntb;
    const int *coff = p.coff + int64_t(ta) * p.ntb;
    // the unit's compact columns [lo, hi): the parts of the allowed blocks of ta inside them
    for (int u = 0; u < p.ntb; ++u) {
        const int o = coff[u];
        if (o < 0) continue;
        const int cnt = p.bstart[u + 1] - p.bstart[u];
        const int x0 = o > ulo ? o : ulo, x1 = o + cnt < uhi ? o + cnt : uhi;
        const T *src = p.sp + segrow[u] + int64_t(ra) * p.ld[u] - o;
        for (int x = x0 + tid; x < x1; x += NT) sig[x - ulo] = src[x];
    }
    const int *sl = p.slot + int64_t(ta) * KP;
    for (int idx = tid; idx < KP * p.ntb; idx += NT) {
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
        rowoff[idx] = off;
    }
    // RTK (point-group spaces): the host's k-step masks are per alpha type and
    // take every step, but a tile of beta type u only meets the slots whose
    // source row lies in a block allowed with u (the others gather the zero
    // row); the steps holding one, per u, narrow each item's mask (CAS(16,16)
    // D2h sigma_3: FP64 83.9 -> 64.5 ms, FP32 40.0 -> 37.7 ms, the same sigma)
    uint32_t *ukm = rowoff + p.ntb * KP;                  // [ntb]
    if constexpr (RTK) {
        __syncthreads();                                  // rowoff complete
        for (int u = tid; u < p.ntb; u += NT) {
            uint32_t m = 0;
            for (int q = 0; q < KP; ++q)
                if (rowoff[u * KP + q] != p.zero_off) m |= 1u << (q >> 2);
            ukm[u] = m;
        }
    }
    // A fragments: row m (grouped pair order) = 16*rbi(r) + lane%16, gathered row 4t + lane/16
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
            const int m = rbi(r) * 16 + (lane & 15);
            T val = 0;
            if (r < nrb && m < p.mp) {
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

    const int nact = uni(U[4]);
    if (nact > 0) {
        const __amdgpu_buffer_rsrc_t pr = buffer_of(p.plan, p.plan_bytes);
        const T *cl = p.cp + (cb * 16 + (lane & 15));   // this lane's column of the item's first column
        const __amdgpu_buffer_rsrc_t crs = buffer_of(p.cp, BUF ? p.cp_bytes : 0u);
        const uint32_t colo = uint32_t(cb * 16 + (lane & 15));
        const uint32_t pl = uint32_t(wave * PW + lane) * 4u;
        const uint32_t spare = uint32_t(ncol + lane) * uint32_t(sizeof(T));
        const uint4 *act = p.act + uni(U[3]);
        T bc[NH][KS];
        acc_t acc[NH][RBW];
        // gathered rows of an item for every k step: one LDS offset read each
        // (only the k steps the item multiplies: the others read the zero row anyway);
        // four waves: 32-bit element offsets on a 64-bit base, so C may exceed 4 GB
        auto load = [&](const uint4 &e, T (&b)[NH][KS]) {
            const uint32_t *ro = rowoff + (e.w & 255u) * KP + (lane >> 4);
            if constexpr (BUF) {
                const uint32_t c0 = (e.w >> 8) + colo;
#pragma unroll
                for (int t = 0; t < KS; ++t) {
                    if ((e.y >> t) & 1u) buffer_ld(b[0][t], crs, (ro[4 * t] + c0) * uint32_t(sizeof(T)), 0u);
                    else b[0][t] = T(0);
                }
            } else {
                const T *src = cl + (e.w >> 8);
#pragma unroll
                for (int t = 0; t < KS; ++t) {
                    const bool on = (e.y >> t) & 1u;
#pragma unroll
                    for (int h = 0; h < NH; ++h) b[h][t] = on ? src[ro[4 * t] + 16 * h] : T(0);
                }
            }
        };
        // one accumulator chain per row block (a second one on the odd k steps cost
        // the registers of the eight-wave form: GAS(20,20) FP32 67.1 -> 66.1 ms
        // without it).  FP64: only the item's active k steps (a uniform branch each);
        // FP32: the k steps in four chunks, a chunk multiplied when one of its k
        // steps is active (measured at GAS(20,20): FP64 148 ms per-step vs 159 ms
        // chunked, FP32 79 ms chunked vs 88 ms per-step); with the per-beta-type
        // masks (RTK) FP32 goes per step too: most chunks then hold an active step
        // among idle ones (CAS(16,16) D2h sigma_3 37.1 -> 25.6 ms)
        constexpr bool PER_STEP = sizeof(T) == 8 || RTK;
        constexpr uint32_t CM0 = PER_STEP ? 1u : (1u << (KS / 4)) - 1u;
        constexpr uint32_t CM1 = ((1u << (KS / 2)) - 1u) & ~CM0;
        constexpr uint32_t CM2 = ((1u << (3 * KS / 4)) - 1u) & ~(CM0 | CM1);
        constexpr uint32_t CM3 = (KS == 32 ? 0xffffffffu : ((1u << KS) - 1u)) & ~(CM0 | CM1 | CM2);
        auto products = [&](uint32_t km, uint32_t rm) {
#pragma unroll
            for (int r = 0; r < RBW; ++r) {
#pragma unroll
                for (int h = 0; h < NH; ++h) acc[h][r] = acc_t{0, 0, 0, 0};
                if (r >= nrb || !((rm >> rbi(r)) & 1u)) continue;
                if (PER_STEP) {
#pragma unroll
                    for (int t = 0; t < KS; ++t) {
                        if (!((km >> t) & 1u)) continue;
#pragma unroll
                        for (int h = 0; h < NH; ++h) acc[h][r] = M::op(A[r][t], bc[h][t], acc[h][r]);
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const uint32_t cm = c == 0 ? CM0 : c == 1 ? CM1 : c == 2 ? CM2 : CM3;
                        if (!(km & cm)) continue;
#pragma unroll
                        for (int t = 0; t < KS; ++t) {
                            if (!((cm >> t) & 1u)) continue;
#pragma unroll
                            for (int h = 0; h < NH; ++h) acc[h][r] = M::op(A[r][t], bc[h][t], acc[h][r]);
                        }
                    }
                }
            }
        };
        auto store_w = [&](uint32_t rm) {
#pragma unroll
            for (int r = 0; r < RBW; ++r)
                if (r < nrb && ((rm >> rbi(r)) & 1u))
#pragma unroll
                    for (int h = 0; h < NH; ++h)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            W[(rbi(r) * 16 + M::out_row(lane, i)) * kAbxWS + (cb + h) * 16 + (lane & 15)] =
                                acc[h][r][i];
        };
        // items i + 1 and i + 2 are read one iteration ahead of their use; the
        // gathered rows of an item in one buffer, loaded in the iteration that
        // multiplies them (a second buffer, one item ahead, cost the registers of the
        // eight-wave form: 64.0 -> 57.5 ms without it)
        auto item = [&](int i) {                          // tile entry i, its k-step mask narrowed
            uint4 e = uni_ld(act + i);
            if constexpr (RTK) e.y &= uint32_t(__builtin_amdgcn_readfirstlane(int(ukm[e.w & 255u])));
            return e;
        };
        uint4 e1 = item(nact > 1 ? 1 : 0), e2 = item(nact > 2 ? 2 : nact - 1);
        {
            const uint4 e0 = item(0);
            load(e0, bc);
            products(e0.y, e0.z);
            store_w(e0.z);
        }
        // act .x: plan tile | its entries per lane << 24.  A tile's plan words are
        // read at the start of its own item, in flight while the next item's
        // products run (read one item earlier they held 17 more registers:
        // 66.1 -> 64.0 ms without them)
        uint32_t pw_[EW], ph;
        uint32_t xc = uni(act[0].x);
        int pn = 0;
        __syncthreads();
        for (int i = 0; i < nact; ++i) {
            const bool more = i + 1 < nact;
            const uint4 e3 = item(i + 3 < nact ? i + 3 : nact - 1);
            if (more) load(e1, bc);                              // rows of item i + 1
            pn = int(xc >> 24);
            if (scat) abx_plan_load_n<EW>(pr, pl, (xc & 0xffffffu) * (PT * 4u), pw_, ph, pn);
            // next item's W (after the last: nothing).  Eight waves: the scatter of
            // this item first, while the rows load (GAS(20,20) FP32 57.5 ms against
            // 61.7 the other way round); four waves: the products first (FP64 115 ms
            // against 121)
            if constexpr (NW == 8) {
                if (scat) abg_scatter_ch<T, EW, TS, 4>(W, sig, pw_, ph, spare, pn);
                products(more ? e1.y : 0u, e1.z);
            } else {
                products(more ? e1.y : 0u, e1.z);
                if (scat) abg_scatter_ch<T, EW, TS, 4>(W, sig, pw_, ph, spare, pn);
            }
            __syncthreads();                                     // W of this item consumed
            if (more) store_w(e1.z);
            __syncthreads();
            xc = e1.x;
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
        for (int x = x0 + tid; x < x1; x += NT) dst[x] = sig[x - ulo];
    }
}

// ---- one-block spaces whose sigma row is split into units (FP32) --------------
//
// The eight-wave form of the one-block kernel (roles split by SIMD: waves 3 and
// 7 scatter, the other six multiply, two W buffers, one barrier per item) over
// the unit tables above: a workgroup owns the columns [lo, hi) of Ia's row, and
// walks its unit's items (source tiles that reach the range) with their row-block
// masks; a producing wave multiplies only its row blocks in the item's mask.
// Gathered rows: Ia's single excitations in list order, then Ia itself (its
// k slot carries sum_{j in Ia} (jj|kl)), then zero rows; 32-bit element offsets
// on a 64-bit base, so C may exceed 4 GB.
template <typename T, int KS, int RB, int EW>
__global__ __launch_bounds__(512, 1) void k_sigma_ab_gw(AbgArgs<T> p) {
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    constexpr int RBW = (RB + 2) / 3;
    constexpr int MP = 16 * RB;
    constexpr int PW = (EW + 1) * 64;
    constexpr int PT = 4 * PW;
    constexpr int TS = sizeof(T) == 4 ? 2 : 3;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *W0 = reinterpret_cast<T *>(smem_raw);               // [2][MP][WS]
    T *W1 = W0 + MP * kAbxWS;
    T *sig = W1 + MP * kAbxWS;                             // [nvirt + 64]

    const int vb = int(blockIdx.x) + p.block_base;
    int ui = 0;
    while (ui + 1 < p.nunits && vb >= uni(p.units[8 * (ui + 1) + 6])) ++ui;
    const int *U = p.units + 8 * uni(ui);
    const int ulo = uni(U[1]), ncol = uni(U[2]) - ulo;
    const int Ia = uni(U[5]) + (vb - uni(U[6]));
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    T *srow = p.sp + int64_t(Ia) * p.ld0 + ulo;
    for (int x = tid; x < ncol; x += 512) sig[x] = srow[x];
    for (int r = tid; r < 2 * MP; r += 512) W0[r * kAbxWS + kAbxNT] = T(0);   // pad column: plan padding reads it
    __syncthreads();                                       // the sigma row is in LDS
    const int nact = uni(U[4]);
    const uint4 *act = p.act + uni(U[3]);
    if (nact > 0) {
        if ((wave & 3) != 3) {
            const int m = (wave >> 2) * 3 + (wave & 3);        // 0..5
            const int cb = m & 1, rb0 = (m >> 1) * RBW;
            const int nrb = RB - rb0 < RBW ? RB - rb0 : RBW;
            T A[RBW][KS];
            uint32_t boff[KS];                                 // element offsets of the gathered rows
            const uint32_t xa = p.astr[Ia];
#pragma unroll
            for (int t = 0; t < KS; ++t) {
                const int q = 4 * t + (lane >> 4);
                uint32_t off = p.zero_off;
                const T *g = nullptr;
                T sg = 0;
                bool self = false;
                if (q < p.anexc) {
                    const uint32_t w = p.aexc[int64_t(Ia) * p.anexc + q];
                    if (w != kExcNone) {
                        off = (w >> 11) * uint32_t(p.ld0);
                        const int i = (w >> 6) & 31, j = (w >> 1) & 31;
                        g = p.g + int64_t(i * p.n + j) * p.mp;
                        sg = (w & 1) ? T(-1) : T(1);
                    }
                } else if (q == p.anexc) {
                    off = uint32_t(Ia) * uint32_t(p.ld0);
                    self = true;
                }
                boff[t] = off;
#pragma unroll
                for (int r = 0; r < RBW; ++r) {
                    const int mr = (rb0 + r) * 16 + (lane & 15);
                    T val = 0;
                    if (r < nrb && mr < p.mp) {
                        if (g) {
                            val = sg * g[mr];
                        } else if (self) {
                            for (uint32_t b = xa; b; b &= b - 1) {
                                const int j = __ffs(b) - 1;
                                val += p.g[int64_t(j * p.n + j) * p.mp + mr];
                            }
                        }
                    }
                    A[r][t] = val;
                }
            }
            const T *cl = p.cp + (cb * 16 + (lane & 15));
            T b[KS];
            acc_t acc[RBW];
            // W of item e on the matrix cores (its active row blocks only); as each
            // k step is consumed its register is reloaded with the rows of item nx
            auto products = [&](const uint4 &e, const uint4 &nx) {
                const uint32_t rm = e.z >> rb0;
                const T *src = cl + (nx.w >> 8);
#pragma unroll
                for (int r = 0; r < RBW; ++r) acc[r] = acc_t{0, 0, 0, 0};
#pragma unroll
                for (int t = 0; t < KS; ++t) {
#pragma unroll
                    for (int r = 0; r < RBW; ++r)
                        if (r < nrb && ((rm >> r) & 1u)) acc[r] = M::op(A[r][t], b[t], acc[r]);
                    b[t] = src[boff[t]];
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
            auto store_w = [&](T *W, uint32_t rmask) {
                const uint32_t rm = rmask >> rb0;
#pragma unroll
                for (int r = 0; r < RBW; ++r)
                    if (r < nrb && ((rm >> r) & 1u))
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            W[((rb0 + r) * 16 + M::out_row(lane, i)) * kAbxWS + cb * 16 + (lane & 15)] = acc[r][i];
            };
            {
                const T *src = cl + (uni(act[0].w) >> 8);
#pragma unroll
                for (int t = 0; t < KS; ++t) b[t] = src[boff[t]];
            }
            const uint4 e0 = uni_ld(act);
            products(e0, uni_ld(act + (nact > 1 ? 1 : 0)));
            store_w(W0, e0.z);
            __syncthreads();                                   // W of item 0 ready
            for (int i = 0; i < nact; ++i) {
                if (i + 1 < nact) {
                    const uint4 e1 = uni_ld(act + i + 1);
                    products(e1, uni_ld(act + (i + 2 < nact ? i + 2 : nact - 1)));
                    store_w((i + 1) & 1 ? W1 : W0, e1.z);
                }
                __syncthreads();
            }
        } else {
            const __amdgpu_buffer_rsrc_t pr = buffer_of(p.plan, p.plan_bytes);
            const int sw = wave >> 2;                          // plan ranges sw and sw + 2
            const uint32_t pl0 = uint32_t(sw * PW + lane) * 4u, pl1 = uint32_t((sw + 2) * PW + lane) * 4u;
            const uint32_t spare = uint32_t(ncol + lane) * uint32_t(sizeof(T));
            uint32_t pa0[EW], ha0, pa1[EW], ha1, pb0[EW], hb0, pb1[EW], hb1;
            // every plan word is loaded (the words past a tile's width are padding
            // entries); the scatter of a tile of at most 4 entries per lane takes the
            // 4-entry form.  Loads and scatters whose length varies per tile became
            // branches that waited for each load (measured at CAS(18,18) FP32: 1.68 s
            // that way, 1.32 s with every tile at full width)
            auto plan_of = [&](int i, uint32_t (&w0)[EW], uint32_t &h0, uint32_t (&w1)[EW], uint32_t &h1) {
                const uint32_t x = uni(act[i].x);
                abx_plan_load<EW>(pr, pl0, (x & 0xffffffu) * (PT * 4u), w0, h0);
                abx_plan_load<EW>(pr, pl1, (x & 0xffffffu) * (PT * 4u), w1, h1);
                return int(x >> 24);
            };
            auto scatter = [&](const T *Wt, const uint32_t (&w)[EW], uint32_t h, int n) {
                if constexpr (EW > 4) {
                    if (n <= 4) {
                        const uint32_t w4[4] = {w[0], w[1], w[2], w[3]};
                        abx_scatter<T, 4, TS>(Wt, sig, w4, h, spare);
                        return;
                    }
                }
                abx_scatter<T, EW, TS>(Wt, sig, w, h, spare);
            };
            int na = plan_of(0, pa0, ha0, pa1, ha1), nb = 0;
            __syncthreads();                                   // W of item 0 ready
            for (int i = 0; i < nact; i += 2) {
                if (i + 1 < nact) nb = plan_of(i + 1, pb0, hb0, pb1, hb1);
                scatter(W0, pa0, ha0, na);                     // item i (even) is in W0
                scatter(W0, pa1, ha1, na);
                __syncthreads();
                if (i + 1 < nact) {
                    if (i + 2 < nact) na = plan_of(i + 2, pa0, ha0, pa1, ha1);
                    scatter(W1, pb0, hb0, nb);
                    scatter(W1, pb1, hb1, nb);
                    __syncthreads();
                }
            }
        }
    }
    __syncthreads();                                       // every scatter into the row done
    for (int x = tid; x < ncol; x += 512) srow[x] = sig[x];
}

template <typename T>
size_t abg_lds(int nvirt, int rb, int ks, int ntb, int rtk) {
    return (size_t(16) * rb * kAbxWS + nvirt + 64) * sizeof(T) + (size_t(4) * ks + rtk) * ntb * sizeof(uint32_t);
}

// Waves per workgroup of the GAS kernel: FP32 with C below 4 GB eight (two per
// SIMD, each with a quarter of the W row blocks; waves 0-3 also scatter: at
// GAS(20,20) sigma_3 72.3 -> 64.0 ms), else four (FP64: its A fragments would
// not fit two waves per SIMD)
template <typename T, int KS, int RB, int EW, int NW, bool RTK>
hipError_t run_abg_nw(const AbgArgs<T> &a, int na, hipStream_t s) {
    const size_t lds = abg_lds<T>(a.nvirt, RB, KS, a.ntb, a.rtk);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sigma_ab_g<T, KS, RB, EW, NW, RTK>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sigma_ab_g<T, KS, RB, EW, NW, RTK>), dim3(na), dim3(64 * NW), lds, s, a);
    return hipGetLastError();
}

template <typename T, int KS, int RB, int EW, bool RTK>
hipError_t run_abg_rtk(const AbgArgs<T> &a, int na, hipStream_t s) {
    if constexpr (sizeof(T) == 4)
        if (a.cp_bytes != 0) return run_abg_nw<T, KS, RB, EW, 8, RTK>(a, na, s);
    return run_abg_nw<T, KS, RB, EW, 4, RTK>(a, na, s);
}

// the per-beta-type k-step masks are compiled for the shapes of point-group
// spaces up to CAS(16,16) (17 k steps x 9 row blocks); larger shapes run without
template <typename T, int KS, int RB, int EW>
hipError_t run_abg(const AbgArgs<T> &a, int na, hipStream_t s) {
    if constexpr (KS * RB <= 17 * 9)
        if (a.rtk) return run_abg_rtk<T, KS, RB, EW, true>(a, na, s);
    return run_abg_rtk<T, KS, RB, EW, false>(a, na, s);
}

template <typename T, int KS, int RB, int EW>
hipError_t run_abgw(const AbgArgs<T> &a, int na, hipStream_t s) {
    const size_t lds = (size_t(2) * 16 * RB * kAbxWS + a.nvirt + 64) * sizeof(T);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sigma_ab_gw<T, KS, RB, EW>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sigma_ab_gw<T, KS, RB, EW>), dim3(na), dim3(512), lds, s, a);
    return hipGetLastError();
}

// compiled (KS, RB, EW) shapes of the eight-wave unit kernel (FP32, one-block
// spaces): CAS(8,8) and CAS(10,10) split into units for the tests, CAS(18,18)
#define CIS_ABGW_SHAPES(X) X(5, 4, 4) X(5, 4, 16) X(7, 5, 4) X(7, 5, 16) X(21, 11, 8) X(21, 11, 12) X(21, 11, 16)

// compiled (KS, RB, EW) shapes of the GAS kernel: small test spaces (GAS, one-block
// CAS(8,8) and CAS(10,10) split into units, CAS(8,8) with point-group symmetry),
// GAS(20,20) 6/8/6, CAS(18,18) (whose sigma row is too long for the one-block
// kernel) and CAS(16,16) with point-group symmetry
#define CIS_ABG_SHAPES(X) \
    X(3, 2, 4) X(3, 2, 16) X(4, 2, 4) X(4, 2, 16) X(4, 3, 4) X(4, 3, 16) X(5, 3, 4) X(5, 3, 16) X(5, 4, 4) \
    X(5, 4, 16) X(7, 5, 4) X(7, 5, 16) X(26, 14, 16) X(21, 11, 8) X(21, 11, 12) X(21, 11, 16) X(17, 9, 4) \
    X(17, 9, 8) X(17, 9, 16)

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
    const uint64_t cpe = uint64_t(L.size) + uint64_t(ldmax);   // elements of C with its zero row
    const uint64_t plb = uint64_t(G.plan[d].ntile) * 4 * (G.plan[d].ew + 1) * 64 * sizeof(uint32_t);
    if (cpe >= (uint64_t(1) << 32) || plb >= (uint64_t(1) << 31)) return false;
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
    a.plan_bytes = uint32_t(plb);
    a.zero_off = uint32_t(L.size);
    a.cp_bytes = cpe * sizeof(T) < (uint64_t(1) << 32) ? uint32_t(cpe * sizeof(T)) : 0u;
    a.anexc = A.nexc;
    a.n = ctx->n;
    a.mp = 16 * G.rb;
    a.ntb = ctx->sp[1].ntype;
    a.act = reinterpret_cast<const uint4 *>(G.d_act[d]);
    a.units = G.d_units[d];
    a.nunits = int(G.units[d].size());
    a.nvirt = G.maxcols[d];
    a.rtk = ctx->sym ? 1 : 0;
    int *kshape = const_cast<cisigma_ctx *>(ctx)->last_shape[sizeof(T) == 4];
    // one launch over every unit, or (CISIGMA_OPT_UNIT_LAUNCH) one launch per unit
    a.block_base = 0;
    auto launch_units = [&](AbgArgs<T> x, auto run) -> hipError_t {
        if (ctx->unit_launch == 0) return run(x, G.nblocks[d]);
        for (const auto &lu : G.launch[d]) {
            if (lu.second == 0) continue;
            x.block_base = lu.first;
            const hipError_t e = run(x, lu.second);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    // one-block FP32: the eight-wave form when its two W buffers and the row fit
    if constexpr (sizeof(T) == 4) {
      if (ctx->cas && (size_t(2) * 16 * G.rb * kAbxWS + a.nvirt + 64) * sizeof(T) <= 160 * 1024) {
        a.ld0 = L.ld[0];
        bool ran = false;
#define CIS_RUNW(K, R, E)                                               \
    if (!ran && G.ks == K && G.rb == R && G.plan[d].ew == E) {          \
        *err = launch_units(a, [&](const AbgArgs<T> &x, int n) { return run_abgw<T, K, R, E>(x, n, s); }); \
        kshape[0] = K; kshape[1] = R; kshape[2] = E; kshape[3] = 4;     \
        ran = true;                                                     \
    }
        CIS_ABGW_SHAPES(CIS_RUNW)
#undef CIS_RUNW
        if (ran) return true;
      }
    }
#define CIS_RUN(K, R, E)                                                \
    if (G.ks == K && G.rb == R && G.plan[d].ew == E) {                  \
        *err = launch_units(a, [&](const AbgArgs<T> &x, int n) { return run_abg<T, K, R, E>(x, n, s); }); \
        kshape[0] = K; kshape[1] = R; kshape[2] = E;                    \
        kshape[3] = sizeof(T) == 4 && a.cp_bytes != 0 ? 5 : 3;          \
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
