// sigma_ss.hip -- same-spin parts sigma_1 (beta-beta) and sigma_2 (alpha-alpha)
// of the sigma vector (Eq. 8).
//
// For one spin with N electrons the same-spin Hamiltonian of Eq. 6 is
//   H_s = sum_pq h_pq a+_p a_q + 1/2 sum_pqrs (pq|rs) a+_p a+_r a_s a_q .
// On N-electron strings the one-electron part equals
//   1/(N-1) sum_pqr h_pq a+_p a+_r a_r a_q   (N >= 2),
// so H_s is one two-body operator, written over ordered pairs P = (p<r),
// Q = (q<s) as
//   H_s = sum_{P,Q} V(P,Q) a+_p a+_r a_s a_q ,   V(P,Q) = T_pqrs - T_psrq,
//   T_pqrs = (pq|rs) + (h_pq d_rs + d_pq h_rs)/(N-1).
// Inserting the (N-2)-electron strings K between creator and annihilator pairs
//   sigma(K+P, :) += e(K,P) sum_Q V(P,Q) e(K,Q) X(K+Q, :)
// where e(K,Q) is the sign of a+_q a+_s |K>.  For each K this is one dense
// product of the (pairs of empty orbitals of K)^2 block of V with the gathered
// rows X(K+Q, :): a matrix-core GEMM, then a row scatter.  X is the CI matrix
// with rows = strings of this spin (C for alpha; C transposed for beta).
//
// N = 1 has no pairs; its one-electron part is applied by k_one_electron.
#include "internal.h"
#include "mfma.h"
#include "bufio.h"

#include <algorithm>
#include <type_traits>

namespace cis {
namespace {


template <typename T>
struct SsArgs {
    const T *X;                 // rows = strings of this spin, padded layout
    T *Y;                       // accumulator, same layout
    const uint32_t *pairs;      // [nK][npv]
    const T *V;                 // [nps][nps]
    const int *stype, *sstart;  // row-spin string types and type starts
    const int64_t *seg;         // [nts][nto]
    const int *ld;              // [nto]
    const int *tile_u, *tile_c0;
    int npv, nK, nps, nto, ntiles;
    // chunk store mode: rows K*npv+P of Ys (row stride ldy) over tiles [tile_begin, tile_end),
    // column c stored at c - col_begin
    T *Ys;
    int64_t ldy;
    int tile_begin, tile_end, col_begin;
    int ysplit;                 // column split of the grid (0: heuristic)
    // row store mode: the product row of pair entry (K, P) for column type u goes to
    // Ys + yoff[K*npv+P] + ycol[type(K+P)][u] (the padded sigma row of K+P)
    const int64_t *yoff;
    const int *ycol;
    const int *klist;           // K of each workgroup (nullptr: K = blockIdx.x)
};

// Workgroup b of n (along x) -> a contiguous range of K per XCD: workgroups are
// dealt to the 8 XCDs in turn, and neighbouring K (in colex order) share many
// of their gathered rows J = K + pair, which then meet in one XCD's L2
// (measured at CAS(16,16): a same-spin pass 9.06 -> 8.91 ms FP32).  A
// permutation of [0, n) for every n.
__device__ __forceinline__ int xcd_contig(int b, int n) {
    const int q = n >> 3, r = n & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// MODE 0: accumulate into Y with atomics; 1: store column chunks of rows
// K*npv+P; 2: store each product row into the row of its pair entry,
// multiplying per item only the k steps and row blocks that hold a gathered
// row or a stored row of the item's column type (GAS: many pairs of a K lead to
// strings not allowed with a given column type; point-group spaces: V is
// block-diagonal by pair irrep, so one column type meets about one pair irrep.
// GAS(20,20) same-spin pass 13.2 -> 7.4 ms FP32, 22.3 -> 12.2 ms FP64; CAS(16,16)
// D2h 5.4 -> 3.5 ms FP32; the same sigma bit for bit)
template <typename T, int KS, int MBL, int MODE>
__global__ __launch_bounds__(256) void k_sigma_ss(SsArgs<T> p) {
    constexpr bool STORE = MODE == 1;
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    using vec_t = typename M::vec_t;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int TW = 16 * VEC;
    constexpr int HALVES = kTileCols / TW;
    constexpr int KP = 4 * KS, MP = 16 * MBL;
    constexpr int NE = KP > MP ? KP : MP;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *As = reinterpret_cast<T *>(smem_raw);            // [MP][KP+1]
    int *rowJ = reinterpret_cast<int *>(As + MP * (KP + 1));
    int *pid = rowJ + NE;
    int *neg = pid + NE;

    // (K in launch order: the XCD-contiguous order of the one-block kernel below
    // made the GAS(20,20) pass slower, 13.9 -> 14.7 ms FP32)
    const int K = p.klist ? p.klist[blockIdx.x] : int(blockIdx.x);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ int any_valid;
    __shared__ unsigned long long colmask;   // column types some row of this K is allowed with
    if (tid == 0) {
        any_valid = 0;
        colmask = 0;
    }
    __syncthreads();
    for (int q = tid; q < NE; q += 256) {
        uint32_t w = (q < p.npv) ? p.pairs[int64_t(K) * p.npv + q] : kPairNone;
        rowJ[q] = (w == kPairNone) ? -1 : int(w >> 11);
        pid[q] = int((w >> 1) & 1023u);
        neg[q] = int(w & 1u);
        if (w != kPairNone) {
            any_valid = 1;
            if (p.nto <= 64) {
                const int t = p.stype[w >> 11];
                unsigned long long m = 0;
                for (int u = 0; u < p.nto; ++u)
                    if (p.seg[int64_t(t) * p.nto + u] >= 0) m |= 1ull << u;
                atomicOr(&colmask, m);
            }
        }
    }
    __syncthreads();
    if (!any_valid) return;
    const unsigned long long cols = p.nto <= 64 ? colmask : ~0ull;
    for (int idx = tid; idx < MP * KP; idx += 256) {
        int P = idx / KP, Q = idx % KP;
        T val = 0;
        if (rowJ[P] >= 0 && rowJ[Q] >= 0) {
            val = p.V[int64_t(pid[P]) * p.nps + pid[Q]];
            if (neg[P] ^ neg[Q]) val = -val;
        }
        As[P * (KP + 1) + Q] = val;
    }
    __syncthreads();
    // The V-block fragments stay in LDS and are read per k step: held in registers
    // (MBL*KS of them) they left one wave per SIMD for the larger pair counts, whose
    // gathers then went unhidden (GAS(20,20) same-spin pass 13.9 -> 13.2 ms FP32,
    // 27.8 -> 22.5 ms FP64 with two waves per SIMD).
    const int a_lane = (lane & 15) * (KP + 1) + (lane >> 4);   // row lane%16, k column lane/16
    int cur_u = -1;
    int64_t boff[KS];     // row offsets of the gathered B rows for the current column type
    int64_t ooff[MBL][4]; // row offsets of the output rows
    uint64_t km = ~0ull;  // MODE 2: k steps and row blocks the current column type uses
    uint32_t rbm = ~0u;
    const int item_end = STORE ? p.tile_end * HALVES : p.ntiles * HALVES;
    for (int item = (STORE ? p.tile_begin * HALVES : 0) + wave + 4 * blockIdx.y; item < item_end;
         item += 4 * gridDim.y) {
        const int tile = item / HALVES;
        const int u = p.tile_u[tile];
        if (!((cols >> (u & 63)) & 1ull)) continue;   // no row of this K lives in column type u
        const int c0 = p.tile_c0[tile] + (item % HALVES) * TW;
        if (u != cur_u) {
            cur_u = u;
#pragma unroll
            for (int t = 0; t < KS; ++t) {
                int J = rowJ[4 * t + (lane >> 4)];
                int64_t o = -1;
                if (J >= 0) {
                    int tj = p.stype[J];
                    int64_t s = p.seg[int64_t(tj) * p.nto + u];
                    if (s >= 0) o = s + int64_t(J - p.sstart[tj]) * p.ld[u];
                }
                boff[t] = o;
            }
#pragma unroll
            for (int rb = 0; rb < MBL; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int P = rb * 16 + M::out_row(lane, i);
                    int J = rowJ[P];
                    int64_t o = -1;
                    if (J >= 0) {
                        int tj = p.stype[J];
                        if (MODE == 2) {
                            const int yc = p.ycol[int64_t(tj) * p.nto + u];
                            const int64_t yo = p.yoff[int64_t(K) * p.npv + P];
                            if (yc >= 0 && yo >= 0) o = yo + yc;
                        } else {
                            int64_t s = p.seg[int64_t(tj) * p.nto + u];
                            if (s >= 0) o = s + int64_t(J - p.sstart[tj]) * p.ld[u];
                        }
                    }
                    ooff[rb][i] = o;
                }
            if constexpr (MODE == 2) {
                km = 0;
#pragma unroll
                for (int t = 0; t < KS; ++t)
                    if (__builtin_amdgcn_ballot_w64(boff[t] >= 0)) km |= 1ull << t;
                rbm = 0;
#pragma unroll
                for (int rb = 0; rb < MBL; ++rb) {
                    const bool any = ooff[rb][0] >= 0 || ooff[rb][1] >= 0 || ooff[rb][2] >= 0 || ooff[rb][3] >= 0;
                    if (__builtin_amdgcn_ballot_w64(any)) rbm |= 1u << rb;
                }
            }
        }
        const int col = c0 + VEC * (lane & 15);
        acc_t acc[MBL][VEC];
#pragma unroll
        for (int rb = 0; rb < MBL; ++rb)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[rb][v] = acc_t{0, 0, 0, 0};
        int ab = a_lane;
        asm volatile("" : "+v"(ab));   // opaque per item: the LDS reads are not hoisted out of the loop
#pragma unroll
        for (int t = 0; t < KS; ++t) {
            if (MODE == 2 && !((km >> t) & 1ull)) continue;
            vec_t b = vec_t{};
            if (boff[t] >= 0) b = *reinterpret_cast<const vec_t *>(p.X + boff[t] + col);
            T a[MBL];
#pragma unroll
            for (int rb = 0; rb < MBL; ++rb) a[rb] = As[ab + rb * 16 * (KP + 1) + 4 * t];
#pragma unroll
            for (int v = 0; v < VEC; ++v)
#pragma unroll
                for (int rb = 0; rb < MBL; ++rb)
                    if (MODE != 2 || ((rbm >> rb) & 1u)) acc[rb][v] = M::op(a[rb], b[v], acc[rb][v]);
        }
        if (STORE) {
            // plain stores: row K*npv + P of the materialised buffer belongs to this workgroup alone
#pragma unroll
            for (int rb = 0; rb < MBL; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int P = rb * 16 + M::out_row(lane, i);
                    if (P >= p.npv) continue;
                    vec_t o;
#pragma unroll
                    for (int v = 0; v < VEC; ++v) o[v] = acc[rb][v][i];
                    *reinterpret_cast<vec_t *>(p.Ys + (int64_t(K) * p.npv + P) * p.ldy + (col - p.col_begin)) = o;
                }
        } else if (MODE == 2) {
            // plain stores: each (pair entry, column) element has one producer
#pragma unroll
            for (int rb = 0; rb < MBL; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (ooff[rb][i] < 0) continue;
                    vec_t o;
#pragma unroll
                    for (int v = 0; v < VEC; ++v) o[v] = acc[rb][v][i];
                    __builtin_nontemporal_store(o, reinterpret_cast<vec_t *>(p.Ys + ooff[rb][i] + col));
                }
        } else {
#pragma unroll
            for (int rb = 0; rb < MBL; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (ooff[rb][i] < 0) continue;
                    T *dst = p.Y + ooff[rb][i] + col;
#pragma unroll
                    for (int v = 0; v < VEC; ++v) unsafeAtomicAdd(dst + v, acc[rb][v][i]);
                }
        }
    }
}

// One-block (CAS) spaces, materialised form: the pair products of one K for the
// columns [col_begin, col_end), stored as rows K*npv + P of Ys (row stride ldy).
// Each wave walks 16*VEC-column items; the gathered rows of its next item are
// loaded while the matrix cores work on the current one.  Missing rows read the
// zero row nstr of X.
template <typename T>
struct SsyArgs {
    const T *X;              // rows = strings of this spin (row stride ld); row nstr is zero
    T *Ys;                   // [nK*npv][ldy]
    const uint32_t *pairs;   // [nK][npv]
    const T *V;              // [nps][nps]
    uint32_t x_bytes;        // bytes of X including the zero row (< 2^31)
    int npv, nK, nps, nstr, ld;
    int64_t ldy;
    int col_begin, col_end;  // multiples of 16*VEC
};

template <typename T, int KS, int MBL>
__global__ __launch_bounds__(256, 2) void k_sigma_ss_y(SsyArgs<T> p) {
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    using vec_t = typename M::vec_t;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int TW = 16 * VEC;
    constexpr int KP = 4 * KS, MP = 16 * MBL;
    constexpr int NE = KP > MP ? KP : MP;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *As = reinterpret_cast<T *>(smem_raw);            // [MP][KP+1]
    int *rowJ = reinterpret_cast<int *>(As + MP * (KP + 1));
    int *pid = rowJ + NE;
    int *neg = pid + NE;

    const int K = xcd_contig(int(blockIdx.x), int(gridDim.x));
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int q = tid; q < NE; q += 256) {
        const uint32_t w = (q < p.npv) ? p.pairs[int64_t(K) * p.npv + q] : kPairNone;
        rowJ[q] = (w == kPairNone) ? -1 : int(w >> 11);
        pid[q] = int((w >> 1) & 1023u);
        neg[q] = int(w & 1u);
    }
    __syncthreads();
    for (int idx = tid; idx < MP * KP; idx += 256) {
        const int P = idx / KP, Q = idx % KP;
        T val = 0;
        if (rowJ[P] >= 0 && rowJ[Q] >= 0) {
            val = p.V[int64_t(pid[P]) * p.nps + pid[Q]];
            if (neg[P] ^ neg[Q]) val = -val;
        }
        As[P * (KP + 1) + Q] = val;
    }
    __syncthreads();
    // V-block fragments read from LDS per k step, as in k_sigma_ss (no spills up to 55 pairs)
    const int a_lane = (lane & 15) * (KP + 1) + (lane >> 4);
    // byte offsets: gathered row of k step t (row 4t + lane/16) and this lane's column
    uint32_t boff[KS];
#pragma unroll
    for (int t = 0; t < KS; ++t) {
        int J = rowJ[4 * t + (lane >> 4)];
        if (J < 0) J = p.nstr;
        boff[t] = (uint32_t(J) * uint32_t(p.ld) + uint32_t(VEC * (lane & 15))) * uint32_t(sizeof(T));
    }
    // byte offsets of this lane's output rows within the K's block of Ys
    uint32_t yoff[MBL][4];
#pragma unroll
    for (int rb = 0; rb < MBL; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            yoff[rb][i] = (uint32_t(rb * 16 + M::out_row(lane, i)) * uint32_t(p.ldy) + uint32_t(VEC * (lane & 15))) *
                          uint32_t(sizeof(T));
    const __amdgpu_buffer_rsrc_t xr = buffer_of(p.X, p.x_bytes);
    const __amdgpu_buffer_rsrc_t yr =
        buffer_of(p.Ys + int64_t(K) * p.npv * p.ldy, uint32_t(int64_t(p.npv) * p.ldy * sizeof(T)));
    const int nitems = (p.col_end - p.col_begin) / TW;
    auto load = [&](int it, vec_t (&b)[KS]) {
        const uint32_t soff = uint32_t(p.col_begin + it * TW) * uint32_t(sizeof(T));
#pragma unroll
        for (int t = 0; t < KS; ++t) buffer_ld(b[t], xr, boff[t], soff);
    };
    auto step = [&](int it, const vec_t (&b)[KS], vec_t (&bn)[KS]) {
        load(it + 4 < nitems ? it + 4 : it, bn);
        __builtin_amdgcn_sched_barrier(0);     // the next item's loads go out first
        acc_t acc[MBL][VEC];
#pragma unroll
        for (int rb = 0; rb < MBL; ++rb)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[rb][v] = acc_t{0, 0, 0, 0};
        int ab = a_lane;
        asm volatile("" : "+v"(ab));   // opaque per item: the LDS reads are not hoisted out of the loop
#pragma unroll
        for (int t = 0; t < KS; ++t) {
            T a[MBL];
#pragma unroll
            for (int rb = 0; rb < MBL; ++rb) a[rb] = As[ab + rb * 16 * (KP + 1) + 4 * t];
#pragma unroll
            for (int v = 0; v < VEC; ++v)
#pragma unroll
                for (int rb = 0; rb < MBL; ++rb) acc[rb][v] = M::op(a[rb], b[t][v], acc[rb][v]);
        }
        const uint32_t soff = uint32_t(it * TW) * uint32_t(sizeof(T));
#pragma unroll
        for (int rb = 0; rb < MBL; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (rb * 16 + M::out_row(lane, i) >= p.npv) continue;
                vec_t o;
#pragma unroll
                for (int v = 0; v < VEC; ++v) o[v] = acc[rb][v][i];
                buffer_st_nt(o, yr, yoff[rb][i], soff);   // each row of Y is read once, by the gather
            }
    };
    if (wave >= nitems) return;
    vec_t b0[KS], b1[KS];
    load(wave, b0);
    for (int it = wave; it < nitems; it += 8) {
        step(it, b0, b1);
        if (it + 4 < nitems) step(it + 4, b1, b0);
    }
}

// out(I, c) = sum over the occupied pairs of I of the materialised rows
// Ys(K*npv + e, c): the owner-computes half of the same-spin part.
template <typename T>
__global__ __launch_bounds__(256) void k_pair_gather(const T *__restrict__ Ys, int64_t ldy, int col_begin,
                                                     int col_end, const int *__restrict__ inv, int per,
                                                     T *__restrict__ out, int64_t ld) {
    using vec_t = typename Mfma<T>::vec_t;
    constexpr int VEC = 16 / sizeof(T);
    __shared__ int rows[64];
    const int I = blockIdx.x;
    for (int q = threadIdx.x; q < per; q += blockDim.x) rows[q] = inv[int64_t(I) * per + q];
    __syncthreads();
    for (int c = col_begin + int(threadIdx.x) * VEC; c < col_end; c += int(blockDim.x) * VEC) {
        // every row of Y is read once (streaming loads); four rows in flight per step
        vec_t acc = vec_t{}, acc2 = vec_t{};
        int q = 0;
        for (; q + 4 <= per; q += 4) {
            const vec_t a0 = __builtin_nontemporal_load(reinterpret_cast<const vec_t *>(Ys + int64_t(rows[q]) * ldy + (c - col_begin)));
            const vec_t a1 = __builtin_nontemporal_load(reinterpret_cast<const vec_t *>(Ys + int64_t(rows[q + 1]) * ldy + (c - col_begin)));
            const vec_t a2 = __builtin_nontemporal_load(reinterpret_cast<const vec_t *>(Ys + int64_t(rows[q + 2]) * ldy + (c - col_begin)));
            const vec_t a3 = __builtin_nontemporal_load(reinterpret_cast<const vec_t *>(Ys + int64_t(rows[q + 3]) * ldy + (c - col_begin)));
            acc += a0 + a1;
            acc2 += a2 + a3;
        }
        for (; q < per; ++q)
            acc += __builtin_nontemporal_load(reinterpret_cast<const vec_t *>(Ys + int64_t(rows[q]) * ldy + (c - col_begin)));
        *reinterpret_cast<vec_t *>(out + int64_t(I) * ld + c) = acc + acc2;
    }
}

// Spaces with several types: out row I (type t) = sum over the occupied pairs
// of I of the stored rows of the pair entries producing I, block by block of
// the column types allowed with t (each row holds the padded blocks of t,
// concatenated in column-type order).  Writes every element of the row.
template <typename T>
__global__ __launch_bounds__(256) void k_pair_gather_rows(const T *__restrict__ Ys, const int64_t *__restrict__ yoff,
                                                          const int *__restrict__ ycol, const int *__restrict__ inv,
                                                          int per, const int *__restrict__ stype,
                                                          const int *__restrict__ sstart, const int64_t *__restrict__ seg,
                                                          const int *__restrict__ ld, int nto, T *__restrict__ out) {
    using vec_t = typename Mfma<T>::vec_t;
    constexpr int VEC = 16 / sizeof(T);
    __shared__ int64_t rows[64];
    const int I = blockIdx.x;
    const int t = stype[I], ri = I - sstart[t];
    for (int q = threadIdx.x; q < per; q += blockDim.x) {
        const int e = inv[int64_t(I) * per + q];
        rows[q] = e >= 0 ? yoff[e] : -1;
    }
    __syncthreads();
    for (int u = 0; u < nto; ++u) {
        const int yc = ycol[int64_t(t) * nto + u];
        if (yc < 0) continue;
        T *dst = out + seg[int64_t(t) * nto + u] + int64_t(ri) * ld[u];
        for (int c = int(threadIdx.x) * VEC; c < ld[u]; c += int(blockDim.x) * VEC) {
            vec_t acc = vec_t{}, acc2 = vec_t{};
            int q = 0;
            for (; q + 2 <= per; q += 2) {
                if (rows[q] >= 0)
                    acc += __builtin_nontemporal_load(reinterpret_cast<const vec_t *>(Ys + rows[q] + yc + c));
                if (rows[q + 1] >= 0)
                    acc2 += __builtin_nontemporal_load(reinterpret_cast<const vec_t *>(Ys + rows[q + 1] + yc + c));
            }
            if (q < per && rows[q] >= 0)
                acc += __builtin_nontemporal_load(reinterpret_cast<const vec_t *>(Ys + rows[q] + yc + c));
            *reinterpret_cast<vec_t *>(dst + c) = acc + acc2;
        }
    }
}

// one-electron same-spin part for strings with a single electron:
// Y(I, :) += h_qq X(I, :) (q the occupied orbital) + sum_{J = a+_l a_q I... } s h_kl X(J, :)
template <typename T>
__global__ __launch_bounds__(256) void k_one_electron(const T *X, T *Y, const uint32_t *exc, int nexc,
                                                      const uint32_t *str, const T *h, int n, const int *stype,
                                                      const int *sstart, const int64_t *seg, const int *ld,
                                                      const int *tile_u, const int *tile_c0, int ntiles, int nto) {
    const int I = blockIdx.x;
    const int ti = stype[I];
    const int ri = I - sstart[ti];
    for (int tile = blockIdx.y; tile < ntiles; tile += gridDim.y) {
        const int u = tile_u[tile];
        const int col = tile_c0[tile] + int(threadIdx.x);
        if (threadIdx.x >= kTileCols) continue;
        int64_t so = seg[int64_t(ti) * nto + u];
        if (so < 0) continue;
        T acc = 0;
        for (uint32_t b = str[I]; b; b &= b - 1) {
            int q = __ffs(b) - 1;
            acc += h[q * n + q] * X[so + int64_t(ri) * ld[u] + col];
        }
        for (int e = 0; e < nexc; ++e) {
            uint32_t w = exc[int64_t(I) * nexc + e];
            if (w == kExcNone) continue;
            int J = int(w >> 11), k = (w >> 6) & 31, l = (w >> 1) & 31;
            int tj = stype[J];
            int64_t s = seg[int64_t(tj) * nto + u];
            if (s < 0) continue;
            T x = X[s + int64_t(J - sstart[tj]) * ld[u] + col];
            acc += ((w & 1) ? -h[k * n + l] : h[k * n + l]) * x;
        }
        Y[so + int64_t(ri) * ld[u] + col] += acc;
    }
}

// Same-spin part for pair counts beyond the compiled MFMA shapes (many empty
// orbitals, few electrons: e.g. 32 orbitals): per K and column, the plain
// double loop Y(K+P) += e(K,P) sum_Q V(P,Q) e(K,Q) X(K+Q), accumulated with
// atomics.  O(nK npv^2) per column; such spaces are small.
template <typename T>
__global__ __launch_bounds__(kTileCols) void k_sigma_ss_direct(SsArgs<T> p) {
    const int K = blockIdx.x;
    const uint32_t *pr = p.pairs + int64_t(K) * p.npv;
    for (int tile = blockIdx.y; tile < p.ntiles; tile += gridDim.y) {
        const int u = p.tile_u[tile];
        const int col = p.tile_c0[tile] + int(threadIdx.x);
        for (int ep = 0; ep < p.npv; ++ep) {
            const uint32_t wp = pr[ep];
            if (wp == kPairNone) continue;
            const int Jp = int(wp >> 11), tp = p.stype[Jp];
            const int64_t sp = p.seg[int64_t(tp) * p.nto + u];
            if (sp < 0) continue;
            const T *vrow = p.V + int64_t((wp >> 1) & 1023u) * p.nps;
            T acc = 0;
            for (int eq = 0; eq < p.npv; ++eq) {
                const uint32_t wq = pr[eq];
                if (wq == kPairNone) continue;
                const int Jq = int(wq >> 11), tq = p.stype[Jq];
                const int64_t sq = p.seg[int64_t(tq) * p.nto + u];
                if (sq < 0) continue;
                const T v = vrow[(wq >> 1) & 1023u];
                const T x = p.X[sq + int64_t(Jq - p.sstart[tq]) * p.ld[u] + col];
                acc += ((wp ^ wq) & 1u) ? -v * x : v * x;
            }
            atomicAdd(&p.Y[sp + int64_t(Jp - p.sstart[tp]) * p.ld[u] + col], acc);
        }
    }
}

template <typename T, int KS, int MBL, int MODE>
hipError_t run_ss(const SsArgs<T> &a, hipStream_t s) {
    constexpr bool STORE = MODE == 1;
    constexpr int KP = 4 * KS, MP = 16 * MBL;
    constexpr int NE = KP > MP ? KP : MP;
    size_t lds = size_t(MP) * (KP + 1) * sizeof(T) + 3 * NE * sizeof(int);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sigma_ss<T, KS, MBL, MODE>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
    constexpr int TW = 16 * (16 / sizeof(T));
    const int items = (STORE ? a.tile_end - a.tile_begin : a.ntiles) * (kTileCols / TW);
    int ysplit = 1;
    while (int64_t(a.nK) * ysplit < 2048 && 4 * ysplit < items) ysplit *= 2;
    if (a.ysplit > 0) ysplit = a.ysplit;
    hipLaunchKernelGGL((k_sigma_ss<T, KS, MBL, MODE>), dim3(a.nK, ysplit), dim3(256), lds, s, a);
    return hipGetLastError();
}

template <typename T, int KS, int MBL>
hipError_t run_ssy(const SsyArgs<T> &a, hipStream_t s) {
    constexpr int KP = 4 * KS, MP = 16 * MBL;
    constexpr int NE = KP > MP ? KP : MP;
    const size_t lds = size_t(MP) * (KP + 1) * sizeof(T) + 3 * NE * sizeof(int);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sigma_ss_y<T, KS, MBL>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sigma_ss_y<T, KS, MBL>), dim3(a.nK), dim3(256), lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch_ssy(const SsyArgs<T> &a, hipStream_t s) {
    const int ks = (a.npv + 3) / 4;
    const int mbl = (a.npv + 15) / 16;
#define CIS_SSY(K, MB) if (ks == K && mbl == MB) return run_ssy<T, K, MB>(a, s);
    CIS_SSY(1, 1) CIS_SSY(2, 1) CIS_SSY(3, 1) CIS_SSY(4, 1) CIS_SSY(4, 2) CIS_SSY(6, 2) CIS_SSY(7, 2) CIS_SSY(9, 3)
    CIS_SSY(12, 3) CIS_SSY(14, 4) CIS_SSY(17, 5) CIS_SSY(20, 5) CIS_SSY(23, 6) CIS_SSY(27, 7) CIS_SSY(30, 8)
    CIS_SSY(34, 9) CIS_SSY(39, 10) CIS_SSY(43, 11)
#undef CIS_SSY
    return hipErrorInvalidValue;
}

// pair counts served by the MFMA kernels: npv = C(m, 2) for m = 2..14 (m =
// empty orbitals + 2; larger m leaves the V block too big for the LDS)
bool ss_shape_compiled(int npv) {
    for (int m = 2; m <= 14; ++m)
        if (npv == m * (m - 1) / 2) return true;
    return npv <= 0;
}

// (KS, MBL) of the compiled pair-kernel shapes, smallest first
#define CIS_SS_SHAPES(X) \
    X(1, 1) X(2, 1) X(3, 1) X(4, 1) X(4, 2) X(6, 2) X(7, 2) X(9, 3) X(12, 3) X(14, 4) X(17, 5) X(20, 5) X(23, 6) \
    X(27, 7) X(30, 8) X(34, 9) X(39, 10) X(43, 11)

template <typename T, int MODE>
hipError_t dispatch_ss_shape(const SsArgs<T> &a, int ks, int mbl, hipStream_t s) {
#define CIS_SSB(K, MB) if (ks == K && mbl == MB) return run_ss<T, K, MB, MODE>(a, s);
    CIS_SS_SHAPES(CIS_SSB)
#undef CIS_SSB
    return hipErrorInvalidValue;
}

template <typename T, int MODE>
hipError_t dispatch_ss(const SsArgs<T> &a, hipStream_t s) {
    const int ks = (a.npv + 3) / 4;
    const int mbl = (a.npv + 15) / 16;
    // (KS, MBL) pairs for npv = C(m, 2), m = empty orbitals + 2
#define CIS_SS(K, MB) if (ks == K && mbl == MB) return run_ss<T, K, MB, MODE>(a, s);
    CIS_SS(1, 1) CIS_SS(2, 1) CIS_SS(3, 1) CIS_SS(4, 1) CIS_SS(4, 2) CIS_SS(6, 2) CIS_SS(7, 2) CIS_SS(9, 3)
    CIS_SS(12, 3) CIS_SS(14, 4) CIS_SS(17, 5) CIS_SS(20, 5) CIS_SS(23, 6) CIS_SS(27, 7) CIS_SS(30, 8)
    CIS_SS(34, 9) CIS_SS(39, 10) CIS_SS(43, 11)
#undef CIS_SS
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t same_spin_t(const cisigma_ctx *ctx, int spin, const void *X, void *Y, void *Ys, int chunk,
                       hipStream_t s) {
    const auto &S = ctx->sp[spin];
    const auto &L = ctx->pl[spin];
    const int other = 1 - spin;
    if (S.nel == 0 || S.nstr == 0) return hipSuccess;
    if (S.nel == 1) {
        const T *h = std::is_same<T, float>::value ? reinterpret_cast<const T *>(ctx->d_h32)
                                                   : reinterpret_cast<const T *>(ctx->d_h64);
        int ysplit = 1;
        while (int64_t(S.nstr) * ysplit < 1024 && ysplit < L.ntiles) ysplit *= 2;
        hipLaunchKernelGGL((k_one_electron<T>), dim3(S.nstr, ysplit), dim3(kTileCols), 0, s,
                           static_cast<const T *>(X), static_cast<T *>(Y), S.d_exc, S.nexc, S.d_str, h, ctx->n,
                           S.d_stype, ctx->d_tstart[spin], L.d_seg, L.d_ld, L.d_tile_u, L.d_tile_c0, L.ntiles,
                           ctx->sp[other].ntype);
        return hipGetLastError();
    }
    SsArgs<T> a{};
    a.X = static_cast<const T *>(X);
    a.Y = static_cast<T *>(Y);
    a.pairs = S.d_pairs;
    a.V = std::is_same<T, float>::value ? reinterpret_cast<const T *>(ctx->d_v32[spin])
                                        : reinterpret_cast<const T *>(ctx->d_v64[spin]);
    a.stype = S.d_stype;
    a.sstart = ctx->d_tstart[spin];
    a.seg = L.d_seg;
    a.ld = L.d_ld;
    a.tile_u = L.d_tile_u;
    a.tile_c0 = L.d_tile_c0;
    a.npv = S.npv;
    a.nK = S.nK;
    a.nps = ctx->nps;
    a.nto = ctx->sp[other].ntype;
    a.ntiles = L.ntiles;
    a.ysplit = ctx->ss_split;
    // spaces with several types: one launch per bucket of K (pairs in the space first)
    auto buckets = [&](auto mode) -> hipError_t {
        constexpr int MODE = decltype(mode)::value;
        for (size_t b = 0; b + 1 < S.bk_start.size(); ++b) {
            SsArgs<T> ab = a;
            ab.klist = S.d_klist + S.bk_start[b];
            ab.nK = S.bk_start[b + 1] - S.bk_start[b];
            if (ab.nK == 0) continue;
            hipError_t e = dispatch_ss_shape<T, MODE>(ab, S.bk_ks[b], S.bk_mbl[b], s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    const bool bucketed = !ctx->cas && S.d_klist != nullptr;
    if (!Ys) {
        if (bucketed) return buckets(std::integral_constant<int, 0>{});
        if (ss_shape_compiled(S.npv)) return dispatch_ss<T, 0>(a, s);
        int ysplit = 1;
        while (int64_t(S.nK) * ysplit < 2048 && ysplit < L.ntiles) ysplit *= 2;
        hipLaunchKernelGGL((k_sigma_ss_direct<T>), dim3(S.nK, ysplit), dim3(kTileCols), 0, s, a);
        return hipGetLastError();
    }
    const int per = S.nel * (S.nel - 1) / 2;
    if (!ctx->cas) {
        // several types: every product row into the row of its pair entry, then the gather
        if (S.ny == 0) return hipErrorInvalidValue;
        a.Ys = static_cast<T *>(Ys);
        a.yoff = S.d_yoff;
        a.ycol = S.d_ycol;
        hipError_t e = bucketed ? buckets(std::integral_constant<int, 2>{}) : dispatch_ss<T, 2>(a, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_pair_gather_rows<T>), dim3(S.nstr), dim3(256), 0, s, static_cast<const T *>(Ys),
                           S.d_yoff, S.d_ycol, S.d_pair_inv, per, S.d_stype, ctx->d_tstart[spin], L.d_seg, L.d_ld,
                           a.nto, static_cast<T *>(Y));
        return hipGetLastError();
    }
    // materialised form, one column chunk at a time: store rows K*npv+P, then gather per string
    const int64_t ld = L.ld[0];
    const uint64_t x_bytes = (uint64_t(S.nstr) + 1) * uint64_t(ld) * sizeof(T);   // the zero row included
    for (int c0 = 0; c0 < ld; c0 += chunk) {
        const int c1 = int(std::min<int64_t>(ld, c0 + chunk));
        hipError_t e;
        if (x_bytes < (uint64_t(1) << 31) && uint64_t(S.npv) * uint64_t(c1 - c0) * sizeof(T) < (uint64_t(1) << 31)) {
            SsyArgs<T> y{};
            y.X = static_cast<const T *>(X);
            y.Ys = static_cast<T *>(Ys);
            y.pairs = S.d_pairs;
            y.V = a.V;
            y.x_bytes = uint32_t(x_bytes);
            y.npv = S.npv;
            y.nK = S.nK;
            y.nps = ctx->nps;
            y.nstr = S.nstr;
            y.ld = int(ld);
            y.ldy = c1 - c0;
            y.col_begin = c0;
            y.col_end = c1;
            e = dispatch_ssy<T>(y, s);
        } else {
            a.Ys = static_cast<T *>(Ys);
            a.ldy = c1 - c0;
            a.col_begin = c0;
            a.tile_begin = c0 / kTileCols;
            a.tile_end = c1 / kTileCols;
            e = dispatch_ss<T, 1>(a, s);
        }
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_pair_gather<T>), dim3(S.nstr), dim3(256), 0, s, static_cast<const T *>(Ys),
                           int64_t(c1 - c0), c0, c1, S.d_pair_inv, per, static_cast<T *>(Y), ld);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_sigma_same_spin(const cisigma_ctx *ctx, int spin, const void *X, void *Y, int dtype,
                                  hipStream_t s, void *Ys, int chunk) {
    return dtype == CISIGMA_FP32 ? same_spin_t<float>(ctx, spin, X, Y, Ys, chunk, s)
                                 : same_spin_t<double>(ctx, spin, X, Y, Ys, chunk, s);
}

bool same_spin_materialisable(int npv) { return ss_shape_compiled(npv); }

bool same_spin_shape_for(int count, int *ks, int *mbl) {
    const int need_k = (count + 3) / 4, need_m = (count + 15) / 16;
    int best = -1;
#define CIS_PICK(K, MB) \
    if (K >= need_k && MB >= need_m && (best < 0 || 16 * MB * 4 * K < best)) { best = 16 * MB * 4 * K; *ks = K; *mbl = MB; }
    CIS_SS_SHAPES(CIS_PICK)
#undef CIS_PICK
    return best >= 0;
}

}  // namespace cis
