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
// Plan entry (32 bits):  bit 31 group start | bits 16..30 target dword index
// (sigma slot x element size / 4) | bits 2..15 W byte offset / 4 | bit 0 sign.
// Padding entries start a group of their own, read W(0, 0) and write the spare
// sigma slot ld.
#include "internal.h"
#include "mfma.h"

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
    int anexc, n, kp, npair, Na, ld;
};

// DPP lane moves (gfx9 controls).  Lanes without a valid source read 0.
constexpr int kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143, kWaveShr1 = 0x138, kWaveShl1 = 0x130;

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

// Exclusive segmented sum across the wave: lane l receives the sum of v over
// lanes j < l back to (and including) the nearest lane j with f != 0.
template <typename T>
__device__ __forceinline__ T wave_segmented_carry(T v, int f) {
#define CIS_SCAN_STEP(CTRL, ROWS)                       \
    {                                                   \
        const T tv = dpp_t<CTRL, ROWS>(v);              \
        const int tf = dpp_i<CTRL, ROWS>(f);            \
        v = f ? v : v + tv;                             \
        f |= tf;                                        \
    }
    CIS_SCAN_STEP(kRowShr + 1, 0xf)
    CIS_SCAN_STEP(kRowShr + 2, 0xf)
    CIS_SCAN_STEP(kRowShr + 4, 0xf)
    CIS_SCAN_STEP(kRowShr + 8, 0xf)
    CIS_SCAN_STEP(kRowBcast15, 0xa)
    CIS_SCAN_STEP(kRowBcast31, 0xc)
#undef CIS_SCAN_STEP
    return dpp_t<kWaveShr1, 0xf>(v);
}

__device__ __forceinline__ float flip_if(float u, uint32_t w) {
    return __int_as_float(__float_as_int(u) ^ int(w << 31));
}
__device__ __forceinline__ double flip_if(double u, uint32_t w) {
    const unsigned long long m = static_cast<unsigned long long>(w & 1u) << 63;
    return __longlong_as_double(static_cast<long long>(static_cast<unsigned long long>(__double_as_longlong(u)) ^ m));
}

// KS: k steps over the gathered rows (4*KS >= anexc+1); RBW: 16-row blocks of
// kl per wave; EW: plan entries per lane and tile.  The four waves are 2 column
// blocks x 2 row-block groups of the 32-column tile.  The gathered-row tile (B)
// and the W tile share one LDS buffer, which keeps a workgroup at ~73 KB for
// CAS(16,16) in FP32 so two workgroups share a CU and one's scatter overlaps the
// other's matrix work.  The next tile's rows and this tile's plan are loaded to
// registers while the matrix cores run.
template <typename T, int KS, int RBW, int EW>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 2 : 1) void k_sigma_ab_x(AbxArgs<T> p) {
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    using vec_t = typename M::vec_t;
    constexpr int KP = 4 * KS;
    constexpr int NT = kAbxNT;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int BS = NT + (sizeof(T) == 4 ? 16 : 0);   // B row stride (bank spread for MFMA reads)
    constexpr int WS = kAbxWS;
    constexpr int MP = 16 * RBW * 2;                       // W rows (>= npair; rows >= npair are zero)
    constexpr int VPR = NT / VEC;                          // 16-byte vectors per gathered row
    constexpr int NPRE = (KP * VPR + 255) / 256;           // prefetched vectors per thread
    constexpr int USZ = KP * BS > MP * WS ? KP * BS : MP * WS;
    constexpr int PT = 4 * EW * 64;                        // plan words per tile
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *U = reinterpret_cast<T *>(smem_raw);                    // B tile, then W tile
    T *sig = U + USZ;                                          // [ld + 1]; slot ld takes the padding entries
    int *jrow = reinterpret_cast<int *>(sig + p.ld + 4);       // [KP]

    const int Ia = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cb = wave & 1, grp = wave >> 1;
    const int64_t rowoff = int64_t(Ia) * p.ld;
    for (int c = tid * VEC; c < p.ld; c += 256 * VEC)
        *reinterpret_cast<vec_t *>(sig + c) = *reinterpret_cast<const vec_t *>(p.sp + rowoff + c);
    if (tid == 0) sig[p.ld] = T(0);
    for (int k = tid; k < KP; k += 256) {
        int J = -1;
        if (k < p.anexc) {
            uint32_t e = p.aexc[int64_t(Ia) * p.anexc + k];
            J = (e == kExcNone) ? -1 : int(e >> 11);
        } else if (k == p.anexc) {
            J = Ia;
        }
        jrow[k] = J;
    }
    // A fragments: row m (kl) = 16*rb + lane%16, column k (gathered row) = 4t + lane/16
    T A[RBW][KS];
    const uint32_t xa = p.astr[Ia];
#pragma unroll
    for (int t = 0; t < KS; ++t) {
        const int k = 4 * t + (lane >> 4);
        const T *g = nullptr;
        T sg = 0;
        if (k < p.anexc) {
            uint32_t e = p.aexc[int64_t(Ia) * p.anexc + k];
            if (e != kExcNone) {
                const int i = (e >> 6) & 31, j = (e >> 1) & 31;   // <Ia|E_ij|Ja>, Ja = Ia - i + j
                g = p.gp + int64_t(i * p.n + j) * p.kp;
                sg = (e & 1) ? T(-1) : T(1);
            }
        }
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
            const int m = (grp * RBW + r) * 16 + (lane & 15);
            T val = 0;
            if (m < p.npair) {
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
    __syncthreads();

    // gathered rows of one tile: vector v -> row v / VPR, columns (v % VPR) * VEC
    auto fetch = [&](int c0, vec_t *buf) {
#pragma unroll
        for (int q = 0; q < NPRE; ++q) {
            const int v = tid + q * 256;
            vec_t x = vec_t{};
            if (v < KP * VPR) {
                const int J = jrow[v / VPR];
                if (J >= 0) x = *reinterpret_cast<const vec_t *>(p.cp + int64_t(J) * p.ld + c0 + (v % VPR) * VEC);
            }
            buf[q] = x;
        }
    };
    auto stash = [&](const vec_t *buf) {
#pragma unroll
        for (int q = 0; q < NPRE; ++q) {
            const int v = tid + q * 256;
            if (v < KP * VPR) *reinterpret_cast<vec_t *>(U + (v / VPR) * BS + (v % VPR) * VEC) = buf[q];
        }
    };
    vec_t bpre[NPRE];
    fetch(0, bpre);
    stash(bpre);
    __syncthreads();

    const char *ub = reinterpret_cast<const char *>(U);
    char *sb = reinterpret_cast<char *>(sig);
    const uint32_t *pw = p.plan + wave * (EW * 64) + lane;
    const int ntile = p.ld / NT;
    for (int tile = 0; tile < ntile; ++tile) {
        const int c0 = tile * NT;
        // ---- in flight during the matrix work: next tile's rows, this tile's plan
        if (tile + 1 < ntile) fetch(c0 + NT, bpre);
        uint32_t ent[EW];
#pragma unroll
        for (int q = 0; q < EW; ++q) ent[q] = pw[int64_t(tile) * PT + q * 64];
        // ---- W = A R on the matrix cores
        acc_t acc[RBW];
#pragma unroll
        for (int r = 0; r < RBW; ++r) acc[r] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < KS; ++t) {
            const T b = U[(4 * t + (lane >> 4)) * BS + cb * 16 + (lane & 15)];
#pragma unroll
            for (int r = 0; r < RBW; ++r) acc[r] = M::op(A[r][t], b, acc[r]);
        }
        __syncthreads();                       // everyone is done reading B
#pragma unroll
        for (int r = 0; r < RBW; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                U[((grp * RBW + r) * 16 + M::out_row(lane, i)) * WS + cb * 16 + (lane & 15)] = acc[r][i];
        __syncthreads();
        // ---- beta-side scatter into the LDS sigma row
        T val[EW], old[EW];
        uint32_t ta[EW];
#pragma unroll
        for (int q = 0; q < EW; ++q) {
            val[q] = flip_if(*reinterpret_cast<const T *>(ub + (ent[q] & 0xfffcu)), ent[q]);
            ta[q] = (ent[q] >> 14) & 0x1fffcu;
            old[q] = *reinterpret_cast<const T *>(sb + ta[q]);
        }
        // entry q ends a group when entry q+1 starts one; the lane's last entry
        // does when the next lane's first one starts a group (the last lane: always)
        const int nx = __builtin_amdgcn_update_dpp(int(0x80000000u), int(ent[0]), kWaveShl1, 0xf, 0xf, false);
        const bool end_last = lane == 63 || nx < 0;
        T run = 0;
        bool seen_end = false, any_start = false;
        uint32_t first_end = 0;
#pragma unroll
        for (int q = 0; q < EW; ++q) {
            const bool st = int(ent[q]) < 0;
            any_start = any_start || st;
            run = st ? val[q] : run + val[q];
            const bool en = (q + 1 < EW) ? int(ent[q + 1]) < 0 : end_last;
            if (en) *reinterpret_cast<T *>(sb + ta[q]) = old[q] + run;
            first_end = (en && !seen_end) ? ta[q] : first_end;
            seen_end = seen_end || en;
        }
        // the group open at the end of each lane continues in the next lanes
        const T carry = wave_segmented_carry<T>(end_last ? T(0) : run, any_start ? 1 : 0);
        if (int(ent[0]) >= 0 && seen_end) {
            T *d = reinterpret_cast<T *>(sb + first_end);
            *d = *d + carry;
        }
        __syncthreads();                       // W consumed
        if (tile + 1 < ntile) stash(bpre);
        __syncthreads();
    }
    for (int cc = tid * VEC; cc < p.ld; cc += 256 * VEC)
        *reinterpret_cast<vec_t *>(p.sp + rowoff + cc) = *reinterpret_cast<const vec_t *>(sig + cc);
}

template <typename T>
size_t abx_lds(int ld, int ks, int rbw) {
    const int KP = 4 * ks, BS = kAbxNT + (sizeof(T) == 4 ? 16 : 0), MP = 32 * rbw;
    const int usz = KP * BS > MP * kAbxWS ? KP * BS : MP * kAbxWS;
    return size_t(usz + ld + 4) * sizeof(T) + KP * sizeof(int);
}

template <typename T, int KS, int RBW, int EW>
hipError_t run_abx(const AbxArgs<T> &a, hipStream_t s) {
    const size_t lds = abx_lds<T>(a.ld, KS, RBW);
    if (lds > 160 * 1024 || 32 * RBW < a.npair || 4 * KS < a.anexc + 1) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sigma_ab_x<T, KS, RBW, EW>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sigma_ab_x<T, KS, RBW, EW>), dim3(a.Na), dim3(256), lds, s, a);
    return hipGetLastError();
}

int ks_of(int anexc) { return (anexc + 1 + 3) / 4; }
int rbw_of(int npair) { return (npair + 31) / 32; }

// The compiled (KS, RBW, EW) shapes: for each (KS, RBW) of the CAS(n, n/2)
// spaces n = 4..16 (and the neighbouring open-shell ones) one plan width sized
// for CAS(n, n/2) and a wider one.
#define CIS_ABX_SHAPES(X)                                                                              \
    X(2, 1, 2) X(2, 1, 16) X(3, 1, 2) X(3, 1, 16) X(4, 1, 4) X(4, 1, 16) X(5, 2, 4) X(5, 2, 16)         \
    X(6, 2, 4) X(6, 2, 16) X(7, 2, 4) X(7, 2, 16) X(8, 3, 6) X(8, 3, 16)                          \
    X(10, 3, 6) X(10, 3, 16) X(11, 3, 8) X(11, 3, 16) X(13, 4, 8) X(13, 4, 16) X(15, 4, 10)            \
    X(15, 4, 16) X(17, 5, 10) X(17, 5, 16)

int width_for(int ks, int rbw, int need) {
    int best = 0;
#define CIS_W(K, R, E) if (ks == K && rbw == R && E >= need && (best == 0 || E < best)) best = E;
    CIS_ABX_SHAPES(CIS_W)
#undef CIS_W
    return best;
}

template <typename T>
bool dispatch_abx(const AbxArgs<T> &a, int ew, hipStream_t s, hipError_t *err) {
    const int ks = ks_of(a.anexc), rbw = rbw_of(a.npair);
#define CIS_RUN(K, R, E) \
    if (ks == K && rbw == R && ew == E) { *err = run_abx<T, K, R, E>(a, s); return true; }
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
    if (abx_lds<T>(x.ld, ks_of(x.anexc), rbw_of(x.npair)) > 160 * 1024) return false;
    return dispatch_abx<T>(x, P.ew, s, err);
}

}  // namespace

int sigma_ab_owner_width(int anexc, int npair, int need) {
    return width_for(ks_of(anexc), rbw_of(npair), need);
}

bool launch_sigma_ab_owner(const cisigma_ctx *ctx, const void *cp, void *sp, int dtype, hipStream_t s,
                           hipError_t *err) {
    return dtype == CISIGMA_FP32 ? owner_t<float>(ctx, cp, sp, s, err) : owner_t<double>(ctx, cp, sp, s, err);
}

}  // namespace cis
