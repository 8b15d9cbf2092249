// sigma_abx.hip -- owner-computes form of the alpha-beta part sigma_3 (Eq. 8)
// for one-block (CAS) spaces of up to 16 orbitals.
//
// One workgroup per output alpha string Ia keeps the whole sigma row of Ia in
// LDS and visits the beta strings in 32-column tiles:
//
//   R(a, Jb)  = C(Ja_a, Jb)        a = the single alpha excitations Ja_a of Ia, plus Ia itself
//   W(kl, Jb) = sum_a A(kl, a) R(a, Jb),  A(kl, a) = s_a (i_a j_a|kl),  A(kl, Ia) = sum_{j in Ia} (jj|kl)
//
// Ia's own row either takes a k slot of the matrix product (SELF) or, when the
// excitations alone fill whole k steps, starts the accumulators as the rank-1
// term A(kl, Ia) C(Ia, Jb) (one k step fewer: 16 instead of 17 at CAS(16,16)).
//   sigma(Ia, Ib) += sum_{(kl, Jb): Ib = E_kl Jb} <Ib|E_kl|Jb> W(kl, Jb)
//
// (kl runs over unordered pairs k >= l: E_kl and E_lk share the integral.)
// The gathered rows R are coalesced row reads of C; W comes from the matrix
// cores; the beta-side scatter stays in LDS, so no global atomics are made and
// every sigma row is written once.
//
// The beta-side scatter goes through a plan built once on the host (abx.h).
#include "internal.h"
#include "mfma.h"
#include "bufio.h"
#include "abx.h"

#include <algorithm>
#include <type_traits>

namespace cis {
namespace {


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


// ---- pieces of the two kernel forms ------------------------------------------
//
// KS: k steps over the gathered rows (4*KS >= anexc+1); RB: 16-row blocks of kl
// (16*RB >= npair); RBW: row blocks per producing wave; EW: plan entries per
// lane and tile.  A producing wave owns one 16-column half of the 32-column
// tile (cb) and a run of row blocks [rb0, rb0 + nrb).

// A(m, Ia) = sum_{j in Ia} (jj|kl) for the kl pair of row m
template <typename T>
__device__ __forceinline__ T abx_self_coef(const AbxArgs<T> &p, uint32_t xa, int m) {
    T val = 0;
    for (uint32_t b = xa; b; b &= b - 1) {
        const int j = __ffs(b) - 1;
        val += p.gp[int64_t(j * p.n + j) * p.kp + m];
    }
    return val;
}

// A fragments of Ia for the wave's row blocks -- row m (kl) = 16*(rb0 + r) +
// lane%16, column k = 4t + lane/16 -- and the byte offsets of the gathered rows
// (missing excitations read the zero row Na).  With SELF, column anexc is Ia's
// own row.
template <typename T, int KS, int RBW, bool SELF>
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
        } else if (SELF && k == p.anexc) {
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
                } else if (SELF && k == p.anexc) {
                    val = abx_self_coef(p, xa, m);
                }
            }
            A[r][t] = val;
        }
    }
}

// Without SELF: A(m, Ia) for the lane's accumulator rows m = 16*(rb0 + r) +
// out_row(lane, i), and the byte offset of C(Ia, column) of the lane's column
template <typename T, int RBW>
__device__ __forceinline__ void abx_self_fragments(const AbxArgs<T> &p, int Ia, int lane, int cb, int rb0, int nrb,
                                                   T (&dI)[RBW][4], uint32_t &boffI) {
    using M = Mfma<T>;
    const uint32_t xa = p.astr[Ia];
#pragma unroll
    for (int r = 0; r < RBW; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = (rb0 + r) * 16 + M::out_row(lane, i);
            dI[r][i] = (r < nrb && m < p.npair) ? abx_self_coef(p, xa, m) : T(0);
        }
    boffI = (uint32_t(Ia) * uint32_t(p.ld) + uint32_t(cb * 16 + (lane & 15))) * uint32_t(sizeof(T));   // < cp_bytes
}

template <typename T, int KS>
__device__ __forceinline__ void abx_load(__amdgpu_buffer_rsrc_t cr, const uint32_t (&boff)[KS], int tile, T (&b)[KS]) {
    const uint32_t soff = uint32_t(tile) * uint32_t(kAbxNT * sizeof(T));
#pragma unroll
    for (int t = 0; t < KS; ++t) buffer_ld(b[t], cr, boff[t], soff);
}

// W = A R on the matrix cores for the rows held in b; as each k step is
// consumed, b[t] is reloaded with the rows of tile `next` (always a valid
// tile), so the loads stay in flight for a whole tile.  Without SELF the
// accumulators start from A(kl, Ia) C(Ia, Jb), cI holding C(Ia, Jb) of this
// tile (reloaded likewise).
template <typename T, int KS, int RBW, bool SELF>
__device__ __forceinline__ void abx_products(__amdgpu_buffer_rsrc_t cr, const T (&A)[RBW][KS],
                                             const uint32_t (&boff)[KS], int next, T (&b)[KS],
                                             typename Mfma<T>::acc_t (&acc)[RBW], const T (&dI)[RBW][4],
                                             uint32_t boffI, T &cI) {
    using M = Mfma<T>;
    const uint32_t soff = uint32_t(next) * uint32_t(kAbxNT * sizeof(T));
    if constexpr (SELF) {
#pragma unroll
        for (int r = 0; r < RBW; ++r) acc[r] = typename M::acc_t{0, 0, 0, 0};
    } else {
#pragma unroll
        for (int r = 0; r < RBW; ++r)
            acc[r] = typename M::acc_t{dI[r][0] * cI, dI[r][1] * cI, dI[r][2] * cI, dI[r][3] * cI};
        buffer_ld(cI, cr, boffI, soff);
    }
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

// ---- eight-wave form with one W buffer (FP64; FP32 where two fit per CU) ---------
//
// The roles are split by SIMD as in the two-buffer form below (waves 3 and 7
// scatter, the other six multiply), but with one W tile: the producing waves
// compute the next tile's W in registers while the scatter waves consume this
// tile's, and store it between two barriers.  The FP64 sigma row leaves room for
// no second tile; in FP32 the smaller LDS lets two workgroups share a compute
// unit (CAS(16,16): 71 KB each, 118 registers), so one workgroup's matrix waves
// issue while the other's wait at a barrier.
template <typename T, int KS, int RB, int EW, bool SELF>
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
    for (int r = tid; r < MP; r += 512) W[r * kAbxWS + kAbxNT] = T(0);   // pad column: plan padding reads it
    const int ntile = p.ld / kAbxNT;
    if ((wave & 3) != 3) {
        const int m = (wave >> 2) * 3 + (wave & 3);        // 0..5
        const int cb = m & 1, rb0 = (m >> 1) * RBW;
        const int nrb = RB - rb0 < RBW ? RB - rb0 : RBW;   // may be <= 0 for small RB
        T A[RBW][KS];
        uint32_t boff[KS];
        abx_fragments<T, KS, RBW, SELF>(p, Ia, lane, cb, rb0, nrb, A, boff);
        T dI[RBW][4] = {};
        uint32_t boffI = 0;
        if constexpr (!SELF) abx_self_fragments<T, RBW>(p, Ia, lane, cb, rb0, nrb, dI, boffI);
        const __amdgpu_buffer_rsrc_t cr = buffer_of(p.cp, p.cp_bytes);
        T b[KS];
        T cI = 0;
        acc_t acc[RBW];
        abx_load<T, KS>(cr, boff, 0, b);
        if constexpr (!SELF) buffer_ld(cI, cr, boffI, 0u);
        abx_products<T, KS, RBW, SELF>(cr, A, boff, ntile > 1 ? 1 : 0, b, acc, dI, boffI, cI);
        __syncthreads();                       // the sigma row is in LDS
        abx_store_w<T, RBW>(W, acc, lane, cb, rb0, nrb);
        __syncthreads();                       // W of tile 0 ready
        for (int tile = 0; tile < ntile; ++tile) {
            if (tile + 1 < ntile) {
                const int t2 = tile + 2 < ntile ? tile + 2 : ntile - 1;
                abx_products<T, KS, RBW, SELF>(cr, A, boff, t2, b, acc, dI, boffI, cI);
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
template <typename T, int KS, int RB, int EW, bool SELF>
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
    for (int r = tid; r < 2 * MP; r += 512) W0[r * kAbxWS + kAbxNT] = T(0);   // pad column: plan padding reads it
    const int ntile = p.ld / kAbxNT;
    __syncthreads();                           // the sigma row is in LDS
    if ((wave & 3) != 3) {
        const int m = (wave >> 2) * 3 + (wave & 3);        // 0..5
        const int cb = m & 1, rb0 = (m >> 1) * RBW;
        const int nrb = RB - rb0 < RBW ? RB - rb0 : RBW;   // may be <= 0 for small RB
        T A[RBW][KS];
        uint32_t boff[KS];
        abx_fragments<T, KS, RBW, SELF>(p, Ia, lane, cb, rb0, nrb, A, boff);
        T dI[RBW][4] = {};
        uint32_t boffI = 0;
        if constexpr (!SELF) abx_self_fragments<T, RBW>(p, Ia, lane, cb, rb0, nrb, dI, boffI);
        const __amdgpu_buffer_rsrc_t cr = buffer_of(p.cp, p.cp_bytes);
        T b[KS];
        T cI = 0;
        acc_t acc[RBW];
        abx_load<T, KS>(cr, boff, 0, b);
        if constexpr (!SELF) buffer_ld(cI, cr, boffI, 0u);
        abx_products<T, KS, RBW, SELF>(cr, A, boff, ntile > 1 ? 1 : 0, b, acc, dI, boffI, cI);
        abx_store_w<T, RBW>(W0, acc, lane, cb, rb0, nrb);
        __syncthreads();                       // W of tile 0 ready
        for (int tile = 0; tile < ntile; ++tile) {
            if (tile + 1 < ntile) {
                const int t2 = tile + 2 < ntile ? tile + 2 : ntile - 1;
                abx_products<T, KS, RBW, SELF>(cr, A, boff, t2, b, acc, dI, boffI, cI);
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

// LDS bytes: nw W tiles and the sigma row with its 64 discard slots
template <typename T>
size_t abx_lds(int ld, int rb, int nw) {
    return (size_t(nw) * 16 * rb * kAbxWS + ld + 64) * sizeof(T);
}

// FP32: the one-W-tile form when two of its workgroups fit on a compute unit
// (registers and LDS, as the runtime's occupancy query reports them): while
// one workgroup waits at a barrier the other's matrix waves issue (CAS(16,16)
// sigma_3 34.6 -> 32.1 ms against the two-W-tile form, which fits one per CU);
// otherwise the two-W-tile form.  FP64: one W tile (its row leaves room for no
// more).  *shared: the one-W-tile form ran two workgroups per CU.  two_w: the
// two-W-tile form in FP32 wherever it fits (CISIGMA_OPT_SIGMA_PATH = 3).
template <typename T, int KS, int RB, int EW, bool SELF>
hipError_t run_abx(const AbxArgs<T> &a, hipStream_t s, int *shared, bool two_w) {
    *shared = 0;
    const size_t lds1 = abx_lds<T>(a.ld, RB, 1);
    if (lds1 > 160 * 1024 || 16 * RB < a.npair || 4 * KS < a.anexc + (SELF ? 1 : 0)) return hipErrorInvalidValue;
    const void *kx = reinterpret_cast<const void *>(&k_sigma_ab_x<T, KS, RB, EW, SELF>);
    hipError_t e = hipFuncSetAttribute(kx, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds1));
    if (e != hipSuccess) return e;
    if constexpr (sizeof(T) == 4) {
        int per_cu = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kx, 512, lds1);
        if (e != hipSuccess) return e;
        const size_t lds2 = abx_lds<T>(a.ld, RB, 2);
        if ((per_cu < 2 || two_w) && lds2 <= 160 * 1024) {
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sigma_ab_ws<T, KS, RB, EW, SELF>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds2));
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_sigma_ab_ws<T, KS, RB, EW, SELF>), dim3(a.Na), dim3(512), lds2, s, a);
            return hipGetLastError();
        }
        *shared = per_cu >= 2 ? 1 : 0;
    }
    hipLaunchKernelGGL((k_sigma_ab_x<T, KS, RB, EW, SELF>), dim3(a.Na), dim3(512), lds1, s, a);
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

// Shapes with Ia's row as the rank-1 start of the accumulators, for the
// CAS(n, n/2) spaces of even n and their neighbours whose excitation count is
// a multiple of 4 (there it saves a k step; elsewhere the row fills padding).
// The 16-entry plan width serves spaces whose target groups would span more
// than four lanes at the narrow width (CAS(8,8), CAS(12,12) and smaller).
#define CIS_ABX_SHAPES_R1(X)                                                                           \
    X(1, 1, 2) X(1, 1, 16) X(2, 2, 2) X(2, 2, 16) X(4, 3, 4) X(4, 3, 16) X(6, 4, 4) X(6, 4, 16)         \
    X(9, 5, 6) X(9, 5, 16) X(12, 7, 8) X(12, 7, 16) X(16, 9, 10) X(16, 9, 16)

int width_for(int ks, int rb, int need) {
    int best = 0;
#define CIS_W(K, R, E) if (ks == K && rb == R && E >= need && (best == 0 || E < best)) best = E;
    CIS_ABX_SHAPES(CIS_W)
#undef CIS_W
    return best;
}

// shape[4] receives {KS, RB, EW, 1: row in a k step, 2: rank-1 start}; *shared, two_w as run_abx
template <typename T>
bool dispatch_abx(const AbxArgs<T> &a, int ew, hipStream_t s, hipError_t *err, int *shape, int *shared,
                  bool two_w) {
    const int rb = rb_of(a.npair);
    if (a.anexc > 0 && a.anexc % 4 == 0) {
        const int ks1 = a.anexc / 4;
#define CIS_RUN1(K, R, E)                                           \
    if (ks1 == K && rb == R && ew == E) {                           \
        *err = run_abx<T, K, R, E, false>(a, s, shared, two_w);     \
        shape[0] = K; shape[1] = R; shape[2] = E; shape[3] = 2;     \
        return true;                                                \
    }
        CIS_ABX_SHAPES_R1(CIS_RUN1)
#undef CIS_RUN1
    }
    const int ks = ks_of(a.anexc);
#define CIS_RUN(K, R, E)                                            \
    if (ks == K && rb == R && ew == E) {                            \
        *err = run_abx<T, K, R, E, true>(a, s, shared, two_w);      \
        shape[0] = K; shape[1] = R; shape[2] = E; shape[3] = 1;     \
        return true;                                                \
    }
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
    if (abx_lds<T>(x.ld, rb_of(x.npair), 1) > 160 * 1024) return false;
    // 32-bit byte offsets of the gathered rows (the zero row Na included) and of the plan
    const uint64_t cpb = (uint64_t(x.Na) + 1) * uint64_t(x.ld) * sizeof(T);
    const uint64_t plb = uint64_t(P.ntile) * 4 * (P.ew + 1) * 64 * sizeof(uint32_t);
    if (cpb >= (uint64_t(1) << 31) || plb >= (uint64_t(1) << 31)) return false;
    x.cp_bytes = uint32_t(cpb);
    x.plan_bytes = uint32_t(plb);
    auto *c = const_cast<cisigma_ctx *>(ctx);
    return dispatch_abx<T>(x, P.ew, s, err, c->last_shape[sizeof(T) == 4], &c->abx_shared[sizeof(T) == 4],
                           ctx->ab_mode == 3);
}

}  // namespace

int sigma_ab_owner_width(int anexc, int npair, int need) {
    return width_for(ks_of(anexc), rb_of(npair), need);
}

bool launch_sigma_ab_owner(const cisigma_ctx *ctx, const void *cp, void *sp, int dtype, hipStream_t s,
                           hipError_t *err) {
    return dtype == CISIGMA_FP32 ? owner_t<float>(ctx, cp, sp, s, err) : owner_t<double>(ctx, cp, sp, s, err);
}

}  // namespace cis
