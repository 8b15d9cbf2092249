// abx.h -- pieces shared by the owner-computes sigma_3 kernels (one-block and
// GAS forms): the tile geometry and the beta-side scatter through a plan.
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
// entry ends its group, else the lane's discard slot (row length + lane) -- in
// bytes for the one-block FP32 kernel, in elements otherwise; bits 0..15: W byte
// offset with the sign in bit 0)
// and a header (bit 0: the lane's first entry starts a group; the rest: where
// the carry from earlier lanes is added).  A group spans at most four lanes, so
// the carry needs three lane shifts.
#pragma once

#include "internal.h"
#include "bufio.h"

namespace cis {

constexpr int kAbxNT = 32;               // tile columns
constexpr int kAbxWS = kAbxNT + 1;       // W row stride

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

// The same for a tile whose plan uses only its first n (1..EW, uniform) entries
// per lane: the others are neither read nor written.
template <typename T, int EW, int TS = (sizeof(T) == 4 ? 0 : 3)>
__device__ __forceinline__ void abx_scatter_n(const T *W, T *sig, const uint32_t (&w)[EW], uint32_t hdr,
                                              uint32_t spare, int n) {
    const char *wb = reinterpret_cast<const char *>(W);
    char *sb = reinterpret_cast<char *>(sig);
    T val[EW], old[EW];
    uint32_t t[EW];
#pragma unroll
    for (int q = 0; q < EW; ++q) {
        if (q >= n) break;
        t[q] = (w[q] >> 16) << TS;
        val[q] = flip_if(*reinterpret_cast<const T *>(wb + (w[q] & 0xfffeu)), w[q]);
        old[q] = *reinterpret_cast<const T *>(sb + t[q]);
    }
    T run = 0;
    bool any_start = (hdr & 1u) != 0;
    uint32_t last = spare;
#pragma unroll
    for (int q = 0; q < EW; ++q) {
        if (q >= n) break;
        const bool st = q == 0 ? (hdr & 1u) != 0 : t[q - 1] != spare;
        any_start = any_start || st;
        run = st ? val[q] : run + val[q];
        *reinterpret_cast<T *>(sb + t[q]) = old[q] + run;
        last = t[q];
    }
    const T tail = last != spare ? T(0) : run;
    const T carry = carry3<T>(tail, any_start ? 1 : 0);
    T *d = reinterpret_cast<T *>(sb + (hdr & ~3u));
    *d = *d + carry;
}

// plan words of the first n entries and the header (the header stays at index EW)
template <int EW>
__device__ __forceinline__ void abx_plan_load_n(__amdgpu_buffer_rsrc_t pr, uint32_t pl, uint32_t soff,
                                                uint32_t (&w)[EW], uint32_t &hdr, int n) {
#pragma unroll
    for (int q = 0; q < EW; ++q)
        if (q < n) w[q] = buffer_ld_u32(pr, pl + q * 256u, soff);
    hdr = buffer_ld_u32(pr, pl + EW * 256u, soff);
}

template <int EW>
__device__ __forceinline__ void abx_plan_load(__amdgpu_buffer_rsrc_t pr, uint32_t pl, uint32_t soff, uint32_t (&w)[EW],
                                              uint32_t &hdr) {
#pragma unroll
    for (int q = 0; q < EW; ++q) w[q] = buffer_ld_u32(pr, pl + q * 256u, soff);
    hdr = buffer_ld_u32(pr, pl + EW * 256u, soff);
}

}  // namespace cis
