// sigma_abx.hip -- owner-computes form of the alpha-beta part sigma_3 (Eq. 8)
// for one-block (CAS) spaces of up to 16 orbitals.
//
// One workgroup per output alpha string Ia keeps the whole sigma row of Ia in
// LDS and visits the beta strings in 32-column tiles:
//
//   R(a, Jb)  = C(Ja_a, Jb)        a = the single alpha excitations Ja_a of Ia, plus Ia itself
//   W(kl, Jb) = sum_a A(kl, a) R(a, Jb),  A(kl, a) = s_a (i_a j_a|kl),  A(kl, Ia) = sum_{j in Ia} (jj|kl)
//   sigma(Ia, Ib) += sum_{(kl, Jb): Ib = E_kl Jb} <Ib|E_kl|Jb> W(kl, Jb)
//
// (kl runs over unordered pairs k >= l: E_kl and E_lk share the integral.)
// The gathered rows R are coalesced row reads of C; W comes from the matrix
// cores; the beta-side scatter stays in LDS, so no global atomics are made and
// every sigma row is written once.
//
// Beta-side scatter plan (identical for every Ia, built once on the host):
// per tile, the (target Ib, W element, sign) contributions sorted by target.
// The sorted list is cut, at target-group boundaries, into one range per wave;
// inside a wave, lane l takes the next EW entries (a group may run over several
// lanes).  Each lane sums its entries group by group and writes every group it
// ends; the part of a group held by earlier lanes arrives through a segmented
// scan across the wave (DPP) and is added to the group's end afterwards.  No
// two lanes write the same target and no wave range splits a group, so the LDS
// read-modify-writes never conflict.
//
// Plan words per wave and tile, lane-interleaved: EW entry words (bits 16..31:
// the sigma slot the entry's running sum goes to -- the group's target when the
// entry ends its group, else the lane's discard slot ld + lane -- in bytes for
// FP32, elements for FP64; bits 0..15: W byte offset with the sign in bit 0)
// and a header (bit 0: the lane's first entry starts a group; the rest: where
// the carry from earlier lanes is added).  A group spans at most four lanes, so
// the carry needs three lane shifts.
#include "internal.h"
#include "mfma.h"
#include "bufio.h"

#include <algorithm>
#include <type_traits>

namespace cis {
namespace {

constexpr int kAbxNT = 32;               // tile columns
constexpr int kAbxWS = kAbxNT + 1;       // W row stride

template <typename T>
struct AbxArgs {
    const T *cp;           // C, alpha-major padded (row stride ld)
    T *sp;                 // sigma accumulator, same layout (read, then overwritten)
    const uint32_t *aexc;  // [Na][anexc]
    const uint32_t *astr;  // [Na]
    const T *gp;           // [n*n][kp]
    const uint32_t *plan;  // [ntile][4 waves][EW][64 lanes]
    uint32_t cp_bytes;     // bytes of C including the zero row (< 2^31)
    uint32_t plan_bytes;   // bytes of the plan (< 2^31)
    int anexc, n, kp, npair, Na, ld;
};


// DPP lane moves (gfx9 controls).  Lanes without a valid source read 0.
constexpr int kWaveShr1 = 0x138;

template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, true);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_t(float v) {
    return __int_as_float(dpp_i<CTRL, ROWS>(__float_as_int(v)));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_t(double v) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = unsigned(dpp_i<CTRL, ROWS>(int(unsigned(b))));
    const unsigned hi = unsigned(dpp_i<CTRL, ROWS>(int(unsigned(b >> 32))));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// u with its sign flipped when bit 0 of w is set
__device__ __forceinline__ float flip_if(float u, uint32_t w) {
    return __int_as_float(__float_as_int(u) ^ int(w << 31));
}
__device__ __forceinline__ double flip_if(double u, uint32_t w) {
    const unsigned long long m = static_cast<unsigned long long>(w & 1u) << 63;
    return __longlong_as_double(static_cast<long long>(static_cast<unsigned long long>(__double_as_longlong(u)) ^ m));
}

// Partial group sums held by the three preceding lanes: lane l receives
// tail(l-1), plus tail(l-2) when lane l-1 has no group boundary, plus tail(l-3)
// when lane l-2 has none either (f: the lane has a group boundary).
template <typename T>
__device__ __forceinline__ T carry3(T tail, int f) {
    const T t1 = dpp_t<kWaveShr1, 0xf>(tail);
    const int f1 = dpp_i<kWaveShr1, 0xf>(f);
    const T t2 = dpp_t<kWaveShr1, 0xf>(t1);
    const int f2 = dpp_i<kWaveShr1, 0xf>(f1);
    const T t3 = dpp_t<kWaveShr1, 0xf>(t2);
    return t1 + (f1 ? T(0) : t2 + (f2 ? T(0) : t3));
}

// ---- pieces of the two kernel forms ------------------------------------------
//
// KS: k steps over the gathered rows (4*KS >= anexc+1); RB: 16-row blocks of kl
// (16*RB >= npair); RBW: row blocks per producing wave; EW: plan entries per
// lane and tile.  A producing wave owns one 16-column half of the 32-column
// tile (cb) and a run of row blocks [rb0, rb0 + nrb).

// A fragments of Ia for the wave's row blocks -- row m (kl) = 16*(rb0 + r) +
// lane%16, column k = 4t + lane/16 -- and the byte offsets of the gathered rows
// (missing excitations read the zero row Na).
template <typename T, int KS, int RBW>
__device__ __forceinline__ void abx_fragments(const AbxArgs<T> &p, int Ia, int lane, int cb, int rb0, int nrb,
                                              T (&A)[RBW][KS], uint32_t (&boff)[KS]) {
    const uint32_t xa = p.astr[Ia];
    const uint32_t col = uint32_t(cb * 16 + (lane & 15));
#pragma unroll
    for (int t = 0; t < KS; ++t) {
        const int k = 4 * t + (lane >> 4);
        int J = p.Na;
        const T *g = nullptr;
        T sg = 0;
        if (k < p.anexc) {
            const uint32_t e = p.aexc[int64_t(Ia) * p.anexc + k];
            if (e != kExcNone) {
                J = int(e >> 11);
                const int i = (e >> 6) & 31, j = (e >> 1) & 31;   // <Ia|E_ij|Ja>, Ja = Ia - i + j
                g = p.gp + int64_t(i * p.n + j) * p.kp;
                sg = (e & 1) ? T(-1) : T(1);
            }
        } else if (k == p.anexc) {
            J = Ia;
        }
        boff[t] = (uint32_t(J) * uint32_t(p.ld) + col) * uint32_t(sizeof(T));   // < cp_bytes
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
            const int m = (rb0 + r) * 16 + (lane & 15);
            T val = 0;
            if (r < nrb && m < p.npair) {
                if (g) {
                    val = sg * g[m];
                } else if (k == p.anexc) {
                    for (uint32_t b = xa; b; b &= b - 1) {
                        const int j = __ffs(b) - 1;
                        val += p.gp[int64_t(j * p.n + j) * p.kp + m];
                    }
                }
            }
            A[r][t] = val;
        }
    }
}

template <typename T, int KS>
__device__ __forceinline__ void abx_load(__amdgpu_buffer_rsrc_t cr, const uint32_t (&boff)[KS], int tile, T (&b)[KS]) {
    const uint32_t soff = uint32_t(tile) * uint32_t(kAbxNT * sizeof(T));
#pragma unroll
    for (int t = 0; t < KS; ++t) buffer_ld(b[t], cr, boff[t], soff);
}

// W = A R on the matrix cores for the rows held in b; as each k step is
// consumed, b[t] is reloaded with the rows of tile `next` (always a valid
// tile), so the loads stay in flight for a whole tile.
template <typename T, int KS, int RBW>
__device__ __forceinline__ void abx_products(__amdgpu_buffer_rsrc_t cr, const T (&A)[RBW][KS],
                                             const uint32_t (&boff)[KS], int next, T (&b)[KS],
                                             typename Mfma<T>::acc_t (&acc)[RBW]) {
    using M = Mfma<T>;
    const uint32_t soff = uint32_t(next) * uint32_t(kAbxNT * sizeof(T));
#pragma unroll
    for (int r = 0; r < RBW; ++r) acc[r] = typename M::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < KS; ++t) {
#pragma unroll
        for (int r = 0; r < RBW; ++r) acc[r] = M::op(A[r][t], b[t], acc[r]);
        buffer_ld(b[t], cr, boff[t], soff);
        __builtin_amdgcn_sched_barrier(0);   // keep the reload next to its k step
    }
}

template <typename T, int RBW>
__device__ __forceinline__ void abx_store_w(T *W, const typename Mfma<T>::acc_t (&acc)[RBW], int lane, int cb,
                                            int rb0, int nrb) {
    using M = Mfma<T>;
#pragma unroll
    for (int r = 0; r < RBW; ++r)
        if (r < nrb)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                W[((rb0 + r) * 16 + M::out_row(lane, i)) * kAbxWS + cb * 16 + (lane & 15)] = acc[r][i];
}

// Beta-side scatter of one tile by one wave; w, hdr: this lane's plan words.
// Every entry writes old + running group sum to its slot (the group's target
// at the group's last entry, the discard slot otherwise), so no two lanes write
// one target and the writes need no branches.
template <typename T, int EW, int TS = (sizeof(T) == 4 ? 0 : 3)>   // TS: log2 of the slot field unit in bytes
__device__ __forceinline__ void abx_scatter(const T *W, T *sig, const uint32_t (&w)[EW], uint32_t hdr,
                                            uint32_t spare) {
    const char *wb = reinterpret_cast<const char *>(W);
    char *sb = reinterpret_cast<char *>(sig);
    T val[EW], old[EW];
    uint32_t t[EW];
#pragma unroll
    for (int q = 0; q < EW; ++q) {
        t[q] = (w[q] >> 16) << TS;
        val[q] = flip_if(*reinterpret_cast<const T *>(wb + (w[q] & 0xfffeu)), w[q]);
        old[q] = *reinterpret_cast<const T *>(sb + t[q]);
    }
    T run = 0;
    bool any_start = (hdr & 1u) != 0;
#pragma unroll
    for (int q = 0; q < EW; ++q) {
        // entry q starts a group when entry q-1 ended one
        const bool st = q == 0 ? (hdr & 1u) != 0 : t[q - 1] != spare;
        any_start = any_start || st;
        run = st ? val[q] : run + val[q];
        *reinterpret_cast<T *>(sb + t[q]) = old[q] + run;
    }
    const T tail = t[EW - 1] != spare ? T(0) : run;   // the part of a group that continues in the next lane
    const T carry = carry3<T>(tail, any_start ? 1 : 0);
    T *d = reinterpret_cast<T *>(sb + (hdr & ~3u));
    *d = *d + carry;
}

template <int EW>
__device__ __forceinline__ void abx_plan_load(__amdgpu_buffer_rsrc_t pr, uint32_t pl, uint32_t soff, uint32_t (&w)[EW],
                                              uint32_t &hdr) {
#pragma unroll
    for (int q = 0; q < EW; ++q) w[q] = buffer_ld_u32(pr, pl + q * 256u, soff);
    hdr = buffer_ld_u32(pr, pl + EW * 256u, soff);
}

// ---- eight-wave form with one W buffer (FP64) ------------------------------------
//
// The roles are split by SIMD as in the FP32 form below (waves 3 and 7 scatter,
// the other six multiply), but the FP64 sigma row leaves room for one W tile
// only: the producing waves compute the next tile's W in registers while the
// scatter waves consume this tile's, and store it between two barriers.
template <typename T, int KS, int RB, int EW>
__global__ __launch_bounds__(512, 1) void k_sigma_ab_x(AbxArgs<T> p) {
    using acc_t = typename Mfma<T>::acc_t;
    using vec_t = typename Mfma<T>::vec_t;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int RBW = (RB + 2) / 3;
    constexpr int MP = 16 * RB;
    constexpr int PW = (EW + 1) * 64;                      // plan words per range and tile
    constexpr int PT = 4 * PW;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *W = reinterpret_cast<T *>(smem_raw);                // [MP][WS]
    T *sig = W + MP * kAbxWS;                              // [ld + 64]: slots ld.. take discarded writes

    const int Ia = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: the roles branch per wave
    const int64_t rowoff = int64_t(Ia) * p.ld;
    for (int c = tid * VEC; c < p.ld; c += 512 * VEC)
        *reinterpret_cast<vec_t *>(sig + c) = *reinterpret_cast<const vec_t *>(p.sp + rowoff + c);
    const int ntile = p.ld / kAbxNT;
    if ((wave & 3) != 3) {
        const int m = (wave >> 2) * 3 + (wave & 3);        // 0..5
        const int cb = m & 1, rb0 = (m >> 1) * RBW;
        const int nrb = RB - rb0 < RBW ? RB - rb0 : RBW;   // may be <= 0 for small RB
        T A[RBW][KS];
        uint32_t boff[KS];
        abx_fragments<T, KS, RBW>(p, Ia, lane, cb, rb0, nrb, A, boff);
        const __amdgpu_buffer_rsrc_t cr = buffer_of(p.cp, p.cp_bytes);
        T b[KS];
        acc_t acc[RBW];
        abx_load<T, KS>(cr, boff, 0, b);
        abx_products<T, KS, RBW>(cr, A, boff, ntile > 1 ? 1 : 0, b, acc);
        __syncthreads();                       // the sigma row is in LDS
        abx_store_w<T, RBW>(W, acc, lane, cb, rb0, nrb);
        __syncthreads();                       // W of tile 0 ready
        for (int tile = 0; tile < ntile; ++tile) {
            if (tile + 1 < ntile) {
                const int t2 = tile + 2 < ntile ? tile + 2 : ntile - 1;
                abx_products<T, KS, RBW>(cr, A, boff, t2, b, acc);
            }
            __syncthreads();                   // W of this tile consumed
            if (tile + 1 < ntile) abx_store_w<T, RBW>(W, acc, lane, cb, rb0, nrb);
            __syncthreads();                   // W of the next tile ready
        }
    } else {
        const __amdgpu_buffer_rsrc_t pr = buffer_of(p.plan, p.plan_bytes);
        const int sw = wave >> 2;                          // plan ranges sw and sw + 2
        const uint32_t pl0 = uint32_t(sw * PW + lane) * 4u, pl1 = uint32_t((sw + 2) * PW + lane) * 4u;
        const uint32_t spare = uint32_t(p.ld + lane) * uint32_t(sizeof(T));
        uint32_t pa0[EW], ha0, pa1[EW], ha1, pb0[EW], hb0, pb1[EW], hb1;
        abx_plan_load<EW>(pr, pl0, 0u, pa0, ha0);
        abx_plan_load<EW>(pr, pl1, 0u, pa1, ha1);
        __syncthreads();                       // the sigma row is in LDS
        __syncthreads();                       // W of tile 0 ready
        for (int tile = 0; tile < ntile; tile += 2) {
            const int t1 = tile + 1 < ntile ? tile + 1 : tile, t2 = tile + 2 < ntile ? tile + 2 : t1;
            abx_plan_load<EW>(pr, pl0, uint32_t(t1) * (PT * 4u), pb0, hb0);
            abx_plan_load<EW>(pr, pl1, uint32_t(t1) * (PT * 4u), pb1, hb1);
            abx_scatter<T, EW>(W, sig, pa0, ha0, spare);
            abx_scatter<T, EW>(W, sig, pa1, ha1, spare);
            __syncthreads();                   // W of this tile consumed
            __syncthreads();                   // W of the next tile ready
            if (tile + 1 < ntile) {
                abx_plan_load<EW>(pr, pl0, uint32_t(t2) * (PT * 4u), pa0, ha0);
                abx_plan_load<EW>(pr, pl1, uint32_t(t2) * (PT * 4u), pa1, ha1);
                abx_scatter<T, EW>(W, sig, pb0, hb0, spare);
                abx_scatter<T, EW>(W, sig, pb1, hb1, spare);
                __syncthreads();
                __syncthreads();
            }
        }
    }
    for (int cc = tid * VEC; cc < p.ld; cc += 512 * VEC)
        *reinterpret_cast<vec_t *>(p.sp + rowoff + cc) = *reinterpret_cast<const vec_t *>(sig + cc);
}

// ---- eight-wave form (FP32): six producing and two scattering waves ----------
//
// On gfx950 an FP32 MFMA keeps its SIMD from issuing vector instructions of
// other waves, so a scatter wave that shares a SIMD with a producing wave waits
// out every matrix instruction.  The roles are therefore split by SIMD: the
// eight waves of a workgroup are placed on the four SIMDs in turn (wave w on
// SIMD w mod 4), waves 3 and 7 scatter (the four plan ranges of a tile, two
// each) and share one SIMD, and the other six multiply -- three 16-row-block
// groups x two 16-column halves -- on the other three SIMDs.  Waves 0-2 and
// 4-6 compute W of tile t+1 into one of two W buffers while waves 3 and 7
// scatter tile t from the other; one barrier per tile.  LDS: two W tiles and
// the sigma row (~88 KB for CAS(16,16)).
template <typename T, int KS, int RB, int EW>
__global__ __launch_bounds__(512, 1) void k_sigma_ab_ws(AbxArgs<T> p) {
    using acc_t = typename Mfma<T>::acc_t;
    using vec_t = typename Mfma<T>::vec_t;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int RBW = (RB + 2) / 3;
    constexpr int MP = 16 * RB;
    constexpr int PW = (EW + 1) * 64;                      // plan words per range and tile
    constexpr int PT = 4 * PW;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *W0 = reinterpret_cast<T *>(smem_raw);               // [2][MP][WS]
    T *W1 = W0 + MP * kAbxWS;
    T *sig = W1 + MP * kAbxWS;                             // [ld + 64]: slots ld.. take discarded writes

    const int Ia = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: the roles branch per wave
    const int64_t rowoff = int64_t(Ia) * p.ld;
    for (int c = tid * VEC; c < p.ld; c += 512 * VEC)
        *reinterpret_cast<vec_t *>(sig + c) = *reinterpret_cast<const vec_t *>(p.sp + rowoff + c);
    const int ntile = p.ld / kAbxNT;
    __syncthreads();                           // the sigma row is in LDS
    if ((wave & 3) != 3) {
        const int m = (wave >> 2) * 3 + (wave & 3);        // 0..5
        const int cb = m & 1, rb0 = (m >> 1) * RBW;
        const int nrb = RB - rb0 < RBW ? RB - rb0 : RBW;   // may be <= 0 for small RB
        T A[RBW][KS];
        uint32_t boff[KS];
        abx_fragments<T, KS, RBW>(p, Ia, lane, cb, rb0, nrb, A, boff);
        const __amdgpu_buffer_rsrc_t cr = buffer_of(p.cp, p.cp_bytes);
        T b[KS];
        acc_t acc[RBW];
        abx_load<T, KS>(cr, boff, 0, b);
        abx_products<T, KS, RBW>(cr, A, boff, ntile > 1 ? 1 : 0, b, acc);
        abx_store_w<T, RBW>(W0, acc, lane, cb, rb0, nrb);
        __syncthreads();                       // W of tile 0 ready
        for (int tile = 0; tile < ntile; ++tile) {
            if (tile + 1 < ntile) {
                const int t2 = tile + 2 < ntile ? tile + 2 : ntile - 1;
                abx_products<T, KS, RBW>(cr, A, boff, t2, b, acc);
                abx_store_w<T, RBW>((tile + 1) & 1 ? W1 : W0, acc, lane, cb, rb0, nrb);
            }
            __syncthreads();
        }
    } else {
        const __amdgpu_buffer_rsrc_t pr = buffer_of(p.plan, p.plan_bytes);
        const int sw = wave >> 2;                          // plan ranges sw and sw + 2
        const uint32_t pl0 = uint32_t(sw * PW + lane) * 4u, pl1 = uint32_t((sw + 2) * PW + lane) * 4u;
        const uint32_t spare = uint32_t(p.ld + lane) * uint32_t(sizeof(T));
        // two tiles per trip, plan words in alternating registers: the words of
        // the next tile stay in flight for a whole tile, across the barrier
        uint32_t pa0[EW], ha0, pa1[EW], ha1, pb0[EW], hb0, pb1[EW], hb1;
        abx_plan_load<EW>(pr, pl0, 0u, pa0, ha0);
        abx_plan_load<EW>(pr, pl1, 0u, pa1, ha1);
        __syncthreads();                       // W of tile 0 ready
        for (int tile = 0; tile < ntile; tile += 2) {
            const int t1 = tile + 1 < ntile ? tile + 1 : tile, t2 = tile + 2 < ntile ? tile + 2 : t1;
            abx_plan_load<EW>(pr, pl0, uint32_t(t1) * (PT * 4u), pb0, hb0);
            abx_plan_load<EW>(pr, pl1, uint32_t(t1) * (PT * 4u), pb1, hb1);
            abx_scatter<T, EW>(W0, sig, pa0, ha0, spare);
            abx_scatter<T, EW>(W0, sig, pa1, ha1, spare);
            __syncthreads();                   // tile consumed; the next W is ready
            if (tile + 1 < ntile) {
                abx_plan_load<EW>(pr, pl0, uint32_t(t2) * (PT * 4u), pa0, ha0);
                abx_plan_load<EW>(pr, pl1, uint32_t(t2) * (PT * 4u), pa1, ha1);
                abx_scatter<T, EW>(W1, sig, pb0, hb0, spare);
                abx_scatter<T, EW>(W1, sig, pb1, hb1, spare);
                __syncthreads();
            }
        }
    }
    for (int cc = tid * VEC; cc < p.ld; cc += 512 * VEC)
        *reinterpret_cast<vec_t *>(p.sp + rowoff + cc) = *reinterpret_cast<const vec_t *>(sig + cc);
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
        // k steps in four chunks; a chunk is multiplied when one of its k steps is active
        constexpr uint32_t CM0 = (1u << (KS / 4)) - 1u;
        constexpr uint32_t CM1 = ((1u << (KS / 2)) - 1u) & ~CM0;
        constexpr uint32_t CM2 = ((1u << (3 * KS / 4)) - 1u) & ~(CM0 | CM1);
        constexpr uint32_t CM3 = (KS == 32 ? 0xffffffffu : ((1u << KS) - 1u)) & ~(CM0 | CM1 | CM2);
        // gathered rows of an item for every k step: one LDS offset read each
        auto load = [&](const uint4 &e, T (&b)[KS]) {
            const uint32_t *ro = rowoff + (e.w & 255u) * KP + (lane >> 4);
            const uint32_t soff = (e.w >> 8) * uint32_t(sizeof(T));
#pragma unroll
            for (int t = 0; t < KS; ++t) buffer_ld(b[t], cr, ro[4 * t] + colb, soff);
        };
        // two accumulators per row block (even and odd k steps): independent MFMA chains
        auto products = [&](uint32_t km, uint32_t rm) {
#pragma unroll
            for (int r = 0; r < RBW; ++r) {
                acc[r] = acc_t{0, 0, 0, 0};
                acc2[r] = acc_t{0, 0, 0, 0};
                if (r >= nrb || !((rm >> (rb0 + r)) & 1u)) continue;
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
        uint32_t pw_[EW], ph, nw_[EW], nh;
        abx_plan_load<EW>(pr, pl, act[0].x * (PT * 4u), pw_, ph);
        __syncthreads();
        for (int i = 0; i < nact; ++i) {
            const bool more = i + 1 < nact;
            const uint4 e3 = act[i + 3 < nact ? i + 3 : nact - 1];
#pragma unroll
            for (int t = 0; t < KS; ++t) bc[t] = bn[t];          // rows of item i + 1
            load(e2, bn);                                        // item i + 2, in flight for a whole item
            abx_plan_load<EW>(pr, pl, e1.x * (PT * 4u), nw_, nh);
            products(more ? e1.y : 0u, e1.z);                    // next item's W (after the last: nothing)
            abx_scatter<T, EW, TS>(W, sig, pw_, ph, spare);
            __syncthreads();                                     // W of this item consumed
            if (more) store_w(e1.z);
            __syncthreads();
#pragma unroll
            for (int q = 0; q < EW; ++q) pw_[q] = nw_[q];
            ph = nh;
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

// compiled (KS, RB, EW) shapes of the GAS kernel: small test spaces and GAS(20,20) 6/8/6
#define CIS_ABG_SHAPES(X) \
    X(3, 2, 4) X(3, 2, 16) X(4, 2, 4) X(4, 2, 16) X(4, 3, 4) X(4, 3, 16) X(26, 14, 16)

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
#define CIS_RUN(K, R, E) \
    if (G.ks == K && G.rb == R && G.plan[d].ew == E) *err = run_abg<T, K, R, E>(a, G.nblocks[d], s);
    CIS_ABG_SHAPES(CIS_RUN)
#undef CIS_RUN
    return true;
}

// LDS bytes: the W tile (two for the eight-wave FP32 form) and the sigma row
// with its 64 discard slots
template <typename T>
size_t abx_lds(int ld, int rb) {
    const size_t nw = sizeof(T) == 4 ? 2 : 1;
    return (nw * 16 * rb * kAbxWS + ld + 64) * sizeof(T);
}

template <typename T, int KS, int RB, int EW>
hipError_t run_abx(const AbxArgs<T> &a, hipStream_t s) {
    const size_t lds = abx_lds<T>(a.ld, RB);
    if (lds > 160 * 1024 || 16 * RB < a.npair || 4 * KS < a.anexc + 1) return hipErrorInvalidValue;
    if constexpr (sizeof(T) == 4) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sigma_ab_ws<T, KS, RB, EW>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_sigma_ab_ws<T, KS, RB, EW>), dim3(a.Na), dim3(512), lds, s, a);
    } else {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sigma_ab_x<T, KS, RB, EW>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_sigma_ab_x<T, KS, RB, EW>), dim3(a.Na), dim3(512), lds, s, a);
    }
    return hipGetLastError();
}

int ks_of(int anexc) { return (anexc + 1 + 3) / 4; }
int rb_of(int npair) { return (npair + 15) / 16; }

// The compiled (KS, RB, EW) shapes: for each (KS, RB) of the CAS(n, n/2)
// spaces n = 4..16 and their open-shell neighbours, the plan width of
// CAS(n, n/2) and a wider one.
#define CIS_ABX_SHAPES(X)                                                                              \
    X(2, 1, 2) X(2, 1, 16) X(3, 2, 2) X(3, 2, 16) X(4, 2, 4) X(4, 2, 16) X(4, 3, 4) X(4, 3, 16)         \
    X(5, 3, 4) X(5, 3, 16) X(6, 3, 4) X(6, 3, 16) X(6, 4, 4) X(6, 4, 16) X(7, 4, 4) X(7, 4, 16)         \
    X(8, 5, 6) X(8, 5, 16) X(10, 5, 6) X(10, 5, 16) X(11, 6, 8) X(11, 6, 16) X(13, 7, 8) X(13, 7, 16)   \
    X(15, 8, 10) X(15, 8, 16) X(17, 9, 10) X(17, 9, 16)

int width_for(int ks, int rb, int need) {
    int best = 0;
#define CIS_W(K, R, E) if (ks == K && rb == R && E >= need && (best == 0 || E < best)) best = E;
    CIS_ABX_SHAPES(CIS_W)
#undef CIS_W
    return best;
}

template <typename T>
bool dispatch_abx(const AbxArgs<T> &a, int ew, hipStream_t s, hipError_t *err) {
    const int ks = ks_of(a.anexc), rb = rb_of(a.npair);
#define CIS_RUN(K, R, E) \
    if (ks == K && rb == R && ew == E) { *err = run_abx<T, K, R, E>(a, s); return true; }
    CIS_ABX_SHAPES(CIS_RUN)
#undef CIS_RUN
    return false;
}

template <typename T>
bool owner_t(const cisigma_ctx *ctx, const void *cp, void *sp, hipStream_t s, hipError_t *err) {
    const ScatterPlan &P = ctx->plan;
    const uint32_t *plan = P.d_entries[sizeof(T) == 4 ? 1 : 0];
    if (!plan || P.ew == 0) return false;
    const auto &A = ctx->sp[0];
    AbxArgs<T> x{};
    x.cp = static_cast<const T *>(cp);
    x.sp = static_cast<T *>(sp);
    x.aexc = A.d_exc;
    x.astr = A.d_str;
    x.gp = std::is_same<T, float>::value ? reinterpret_cast<const T *>(ctx->d_gp32)
                                         : reinterpret_cast<const T *>(ctx->d_gp64);
    x.plan = plan;
    x.anexc = A.nexc;
    x.n = ctx->n;
    x.kp = ctx->kp;
    x.npair = ctx->npair;
    x.Na = A.nstr;
    x.ld = ctx->pl[0].ld[0];
    if (abx_lds<T>(x.ld, rb_of(x.npair)) > 160 * 1024) return false;
    // 32-bit byte offsets of the gathered rows (the zero row Na included) and of the plan
    const uint64_t cpb = (uint64_t(x.Na) + 1) * uint64_t(x.ld) * sizeof(T);
    const uint64_t plb = uint64_t(P.ntile) * 4 * (P.ew + 1) * 64 * sizeof(uint32_t);
    if (cpb >= (uint64_t(1) << 31) || plb >= (uint64_t(1) << 31)) return false;
    x.cp_bytes = uint32_t(cpb);
    x.plan_bytes = uint32_t(plb);
    return dispatch_abx<T>(x, P.ew, s, err);
}

}  // namespace

int sigma_ab_gas_width(int ks, int rb, int need) { return gas_width_for(ks, rb, need); }

bool launch_sigma_ab_gas(const cisigma_ctx *ctx, const void *cp, void *sp, int dtype, hipStream_t s,
                         hipError_t *err) {
    return dtype == CISIGMA_FP32 ? gas_t<float>(ctx, cp, sp, s, err) : gas_t<double>(ctx, cp, sp, s, err);
}

int sigma_ab_owner_width(int anexc, int npair, int need) {
    return width_for(ks_of(anexc), rb_of(npair), need);
}

bool launch_sigma_ab_owner(const cisigma_ctx *ctx, const void *cp, void *sp, int dtype, hipStream_t s,
                           hipError_t *err) {
    return dtype == CISIGMA_FP32 ? owner_t<float>(ctx, cp, sp, s, err) : owner_t<double>(ctx, cp, sp, s, err);
}

}  // namespace cis
