// davidson.hip -- Davidson eigensolver around sigma = H C (Sec. 2.1; Sec. 3.3
// steps 1-4):
//   (1) initial subspace: unit vectors on the lowest diagonal elements, their
//       sigma vectors, diagonalisation of the projected matrix G = B^T H B;
//   (2) preconditioner: the diagonal H_II;
//   (3) correction t = r / (theta - H_II) for each unconverged root, made
//       orthogonal to all previous vectors (classical Gram-Schmidt, twice);
//   (4) sigma of the new vectors, updated G, re-diagonalisation; repeat.
// When the basis would exceed max_space it collapses onto the current Ritz
// vectors together with the part of the previous iteration's Ritz vectors
// outside them (a thick restart, which keeps the direction the iteration was
// moving in), or onto the current Ritz vectors alone.  Vector arithmetic runs in HIP kernels with FP64 accumulation;
// only the projected matrix (max_space^2 doubles) and a few norms cross to the
// host each iteration.  The projected eigenproblem is solved on the host
// (Householder tridiagonalisation and implicit QL, symeig.h).
//
// Mixed precision (FP32 basis and sigma): whenever the FP32 iteration meets
// the convergence test (and, if refine_every > 0, every refine_every
// iterations), the Ritz vectors are formed in FP64, their sigma is rebuilt in
// FP64, and the basis collapses onto them with the FP64 sigma (iterative
// refinement).  Convergence is only
// declared there, on FP64 residual norms, and the returned energies are the
// FP64 Rayleigh quotients.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <functional>
#include <type_traits>
#include <vector>

#include "internal.h"
#include "symeig.h"

namespace cis {
namespace {

constexpr int kRedBlocks = 1024;
constexpr int kRitzRoots = 4;     // roots per pass of the batched Ritz kernel
constexpr int kGroup = 8;
constexpr int kMultiY = 4;        // vectors per pass of the blocked dot / update kernels
constexpr int kThick = 16;        // most vectors kept by a thick restart (current + previous Ritz vectors)

template <typename T>
__device__ __forceinline__ double ld(const T *p, int64_t i) { return double(p[i]); }

// Element access of the streaming kernels.  Quad form (Q, for vectors whose
// length and stride are multiples of 4): each thread owns four consecutive
// elements and moves them with 16-byte loads and stores, which keeps about
// twice the bytes in flight of four-byte accesses (measured: a Ritz-shaped pass
// over 20 FP32 vectors streams at 4.7 TB/s this way against 2.2 TB/s).  Plain
// form: E elements blockDim apart, bounds-checked against N.
template <bool Q, int E>
struct Lanes {
    static_assert(!Q || E == 4, "the quad form moves four elements");
    __device__ static int64_t start() {
        return Q ? (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) * 4
                 : int64_t(blockIdx.x) * blockDim.x * E + threadIdx.x;
    }
    __device__ static int64_t stride() { return int64_t(gridDim.x) * blockDim.x * E; }
    __device__ static int64_t at(int64_t n0, int u) { return Q ? n0 + u : n0 + int64_t(u) * blockDim.x; }
};

__device__ __forceinline__ void ld4(const float *p, double (&o)[4]) {
    const float4 v = *reinterpret_cast<const float4 *>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void ld4(const double *p, double (&o)[4]) {
    const double2 a = reinterpret_cast<const double2 *>(p)[0], b = reinterpret_cast<const double2 *>(p)[1];
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}
__device__ __forceinline__ void st4(float *p, const double (&v)[4]) {
    *reinterpret_cast<float4 *>(p) = make_float4(float(v[0]), float(v[1]), float(v[2]), float(v[3]));
}
__device__ __forceinline__ void st4(double *p, const double (&v)[4]) {
    reinterpret_cast<double2 *>(p)[0] = make_double2(v[0], v[1]);
    reinterpret_cast<double2 *>(p)[1] = make_double2(v[2], v[3]);
}

// o[u] = p[element u of the thread's group at n0] (0 beyond N in the plain form)
template <bool Q, int E, typename T>
__device__ __forceinline__ void lde(const T *p, int64_t n0, int64_t N, double (&o)[E]) {
    if constexpr (Q) {
        ld4(p + n0, o);
    } else {
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int64_t n = Lanes<Q, E>::at(n0, u);
            o[u] = n < N ? double(p[n]) : 0.0;
        }
    }
}

// the same in the storage type (converted where used, which keeps FP32 operands
// in half the registers)
__device__ __forceinline__ void ld4t(const float *p, float (&o)[4]) {
    const float4 v = *reinterpret_cast<const float4 *>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void ld4t(const double *p, double (&o)[4]) {
    const double2 a = reinterpret_cast<const double2 *>(p)[0], b = reinterpret_cast<const double2 *>(p)[1];
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}

template <bool Q, int E, typename T>
__device__ __forceinline__ void lde_t(const T *p, int64_t n0, int64_t N, T (&o)[E]) {
    if constexpr (Q) {
        ld4t(p + n0, o);
    } else {
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int64_t n = Lanes<Q, E>::at(n0, u);
            o[u] = n < N ? p[n] : T(0);
        }
    }
}

template <bool Q, int E, typename T>
__device__ __forceinline__ void ste(T *p, int64_t n0, int64_t N, const double (&v)[E]) {
    if constexpr (Q) {
        st4(p + n0, v);
        (void)N;
    } else {
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int64_t n = Lanes<Q, E>::at(n0, u);
            if (n < N) p[n] = T(v[u]);
        }
    }
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < int(blockDim.x >> 6); ++i) s += sh[i];
    return s;
}

// partial[b][i] = sum over block b's slice of X_i . y
template <typename TX, typename TY>
__global__ __launch_bounds__(256) void k_dots(const TX *X, int64_t sx, int nx, const TY *y, int64_t N,
                                              double *partial) {
    __shared__ double sh[8];
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int i0 = 0; i0 < nx; i0 += kGroup) {
        double acc[kGroup];
#pragma unroll
        for (int j = 0; j < kGroup; ++j) acc[j] = 0;
        for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < N; n += stride) {
            double yv = double(y[n]);
#pragma unroll
            for (int j = 0; j < kGroup; ++j)
                if (i0 + j < nx) acc[j] += double(X[(i0 + j) * sx + n]) * yv;
        }
#pragma unroll
        for (int j = 0; j < kGroup; ++j) {
            if (i0 + j >= nx) break;
            double s = block_sum(acc[j], sh);
            if (threadIdx.x == 0) partial[int64_t(blockIdx.x) * nx + i0 + j] = s;
        }
    }
}

// partial[b][j * nx + i] = sum over block b's slice of X_i . Y_j, for j < ny <= kMultiY:
// X is read once for all Y
template <typename TX, typename TY, bool Q>
__global__ __launch_bounds__(256) void k_dots_multi(const TX *X, int64_t sx, int nx, const TY *Y, int64_t sy, int ny,
                                                    int64_t N, double *partial) {
    // X vectors per pass over Y (four in the FP64 quad form: its accumulators and
    // loads of eight would leave fewer than four waves per SIMD for the 1,024
    // workgroups; operands stay in their storage type until used)
    constexpr int GX = Q && sizeof(TX) == 8 ? 4 : 8;
    constexpr int E = Q ? 4 : 1;
    using L = Lanes<Q, E>;
    __shared__ double sh[4][GX * kMultiY];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int i0 = 0; i0 < nx; i0 += GX) {
        double acc[GX][kMultiY];
#pragma unroll
        for (int a = 0; a < GX; ++a)
#pragma unroll
            for (int j = 0; j < kMultiY; ++j) acc[a][j] = 0;
        for (int64_t n0 = L::start(); n0 < N; n0 += L::stride()) {
            TY yv[kMultiY][E];
#pragma unroll
            for (int j = 0; j < kMultiY; ++j) {
                if (j < ny) {
                    lde_t<Q, E>(Y + j * sy, n0, N, yv[j]);
                } else {
#pragma unroll
                    for (int e = 0; e < E; ++e) yv[j][e] = TY(0);
                }
            }
#pragma unroll
            for (int a = 0; a < GX; ++a) {
                if (i0 + a >= nx) break;
                TX xv[E];
                lde_t<Q, E>(X + (i0 + a) * sx, n0, N, xv);
#pragma unroll
                for (int j = 0; j < kMultiY; ++j)
#pragma unroll
                    for (int e = 0; e < E; ++e) acc[a][j] += double(xv[e]) * double(yv[j][e]);
            }
        }
#pragma unroll
        for (int a = 0; a < GX; ++a)
#pragma unroll
            for (int j = 0; j < kMultiY; ++j) {
                double v = acc[a][j];
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
                if (l == 0) sh[w][a * kMultiY + j] = v;
            }
        __syncthreads();
        if (threadIdx.x < GX * kMultiY) {
            const int a = threadIdx.x / kMultiY, j = threadIdx.x % kMultiY;
            const double v = sh[0][threadIdx.x] + sh[1][threadIdx.x] + sh[2][threadIdx.x] + sh[3][threadIdx.x];
            if (i0 + a < nx && j < ny) partial[int64_t(blockIdx.x) * nx * ny + j * nx + i0 + a] = v;
        }
        __syncthreads();
    }
}

// T_j -= sum_i c[j * nx + i] X_i for j < ny <= kMultiY: X is read once for all T_j
template <typename T>
__global__ __launch_bounds__(256) void k_subtract_multi(const T *X, int64_t sx, int nx, const double *c, int ny,
                                                        T *Tv, int64_t st, int64_t N) {
    __shared__ double cs[kMultiY * 512];
    for (int i = threadIdx.x; i < ny * nx; i += blockDim.x) cs[i] = c[i];
    __syncthreads();
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < N; n += stride) {
        double v[kMultiY];
#pragma unroll
        for (int j = 0; j < kMultiY; ++j) v[j] = j < ny ? double(Tv[j * st + n]) : 0.0;
#pragma unroll 8
        for (int i = 0; i < nx; ++i) {
            const double xv = double(X[i * sx + n]);
#pragma unroll
            for (int j = 0; j < kMultiY; ++j) v[j] -= cs[j * nx + i] * xv;
        }
#pragma unroll
        for (int j = 0; j < kMultiY; ++j)
            if (j < ny) Tv[j * st + n] = T(v[j]);
    }
}

// T_j -= sum_i c[j * nx + i] X_i for j < NY (one pass over X, as k_subtract_multi), with
// per-block partial sums of |T_j|^2 before the update and of T_j . T_k (k <= j)
// of the stored (rounded) results: partial[b][v], v < NY + NY(NY+1)/2
template <typename T, int NY, bool Q>
__global__ __launch_bounds__(256) void k_subtract_gram(const T *X, int64_t sx, int nx, const double *c, T *Tv,
                                                       int64_t st, int64_t N, double *partial) {
    constexpr int NV = NY + NY * (NY + 1) / 2;
    constexpr int E = Q ? 4 : 1;
    using L = Lanes<Q, E>;
    __shared__ double cs[NY * 512];
    __shared__ double sh[4][NV];
    for (int i = threadIdx.x; i < NY * nx; i += blockDim.x) cs[i] = c[i];
    __syncthreads();
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0;
    for (int64_t n0 = L::start(); n0 < N; n0 += L::stride()) {
        double v[NY][E];
#pragma unroll
        for (int j = 0; j < NY; ++j) {
            lde<Q, E>(Tv + j * st, n0, N, v[j]);
#pragma unroll
            for (int e = 0; e < E; ++e) acc[j] += v[j][e] * v[j][e];
        }
#pragma unroll 8
        for (int i = 0; i < nx; ++i) {
            double xv[E];
            lde<Q, E>(X + i * sx, n0, N, xv);
#pragma unroll
            for (int j = 0; j < NY; ++j)
#pragma unroll
                for (int e = 0; e < E; ++e) v[j][e] -= cs[j * nx + i] * xv[e];
        }
        double u[NY][E];
#pragma unroll
        for (int j = 0; j < NY; ++j) {
#pragma unroll
            for (int e = 0; e < E; ++e) u[j][e] = double(T(v[j][e]));
            ste<Q, E>(Tv + j * st, n0, N, u[j]);
        }
        int q = NY;
#pragma unroll
        for (int j = 0; j < NY; ++j)
#pragma unroll
            for (int k = 0; k <= j; ++k, ++q)
#pragma unroll
                for (int e = 0; e < E; ++e) acc[q] += u[j][e] * u[k][e];
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double x = acc[v];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (l == 0) sh[w][v] = x;
    }
    __syncthreads();
    if (threadIdx.x < NV)
        partial[int64_t(blockIdx.x) * NV + threadIdx.x] =
            sh[0][threadIdx.x] + sh[1][threadIdx.x] + sh[2][threadIdx.x] + sh[3][threadIdx.x];
}

// D_j = sum_{k < NY} w[j * NY + k] T_k for j < nd (FP64 combination, one rounding)
template <typename T, int NY, bool Q>
__global__ __launch_bounds__(256) void k_combine_new(const T *Tv, int64_t st, const double *w, int nd, T *D,
                                                     int64_t sd, int64_t N) {
    constexpr int E = Q ? 4 : 1;
    using L = Lanes<Q, E>;
    __shared__ double ws[NY * NY];
    for (int i = threadIdx.x; i < nd * NY; i += blockDim.x) ws[i] = w[i];
    __syncthreads();
    for (int64_t n0 = L::start(); n0 < N; n0 += L::stride()) {
        double t[NY][E];
#pragma unroll
        for (int k = 0; k < NY; ++k) lde<Q, E>(Tv + k * st, n0, N, t[k]);
        for (int j = 0; j < nd; ++j) {
            double a[E];
#pragma unroll
            for (int e = 0; e < E; ++e) a[e] = 0;
#pragma unroll
            for (int k = 0; k < NY; ++k)
#pragma unroll
                for (int e = 0; e < E; ++e) a[e] += ws[j * NY + k] * t[k][e];
            ste<Q, E>(D + j * sd, n0, N, a);
        }
    }
}

// out[i] = sum over the nb blocks of partial[b][i]: one wave per output
__global__ __launch_bounds__(64) void k_reduce_partials(const double *partial, int nb, int nx, double *out) {
    const int i = blockIdx.x;
    if (i >= nx) return;
    double s = 0;
    for (int b = int(threadIdx.x); b < nb; b += 64) s += partial[int64_t(b) * nx + i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (threadIdx.x == 0) out[i] = s;
}

// Ritz vectors, their sigma, residual-norm partials and preconditioned
// corrections of up to R roots in one pass over the basis (B and S are read
// once for all roots).  y: [nr][m] root-major coefficients, theta: [nr].
// (WX: also write the Ritz vectors and their sigma.  R = the roots of the pass, so
// the accumulators fit in 128 registers: four waves per SIMD keep the 1,024
// workgroups of a pass resident at once; at 133 registers a quarter of them ran
// as a second round and the pass took ~1.6x)
template <typename T, int R, bool WX, bool Q>
__global__ __launch_bounds__(256) void k_ritz_multi(const T *B, const T *S, int64_t sv, int m, int nr,
                                                    const double *y, const double *theta, const double *hd,
                                                    double *xout, T *sout, T *tout, int64_t N, double *partial) {
    __shared__ double sh[8];
    __shared__ double ys[R][512];
    __shared__ double th[R];
    for (int i = threadIdx.x; i < R * m; i += blockDim.x) ys[i / m][i % m] = (i / m) < nr ? y[i] : 0.0;
    if (threadIdx.x < R) th[threadIdx.x] = threadIdx.x < nr ? theta[threadIdx.x] : 0.0;
    __syncthreads();
    double rr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) rr[r] = 0;
    // U elements per thread (consecutive in the quad form, else blockDim apart):
    // two basis vectors' loads in flight
    constexpr int U = 4;
    using L = Lanes<Q, U>;
    for (int64_t n0 = L::start(); n0 < N; n0 += L::stride()) {
        double x[R][U], s[R][U];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int u = 0; u < U; ++u) x[r][u] = s[r][u] = 0;
#pragma unroll 2
        for (int i = 0; i < m; ++i) {
            double b[U], c[U];
            lde<Q, U>(B + i * sv, n0, N, b);
            lde<Q, U>(S + i * sv, n0, N, c);
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    x[r][u] += ys[r][i] * b[u];
                    s[r][u] += ys[r][i] * c[u];
                }
        }
        double h[U];
        lde<Q, U>(hd, n0, N, h);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r >= nr) break;
            double t[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // beyond N (plain form) x = s = 0: a zero residual and correction
                const double res = s[r][u] - th[r] * x[r][u];
                rr[r] += res * res;
                double dd = th[r] - h[u];
                if (fabs(dd) < 1e-8) dd = dd < 0 ? -1e-8 : 1e-8;
                t[u] = res / dd;
            }
            ste<Q, U>(tout + r * N, n0, N, t);
            if (WX) {                          // the Ritz vectors and their sigma: only when asked
                ste<Q, U>(xout + r * N, n0, N, x[r]);
                ste<Q, U>(sout + r * N, n0, N, s[r]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double tot = block_sum(rr[r], sh);
        if (threadIdx.x == 0 && r < nr) partial[int64_t(r) * gridDim.x + blockIdx.x] = tot;
        __syncthreads();
    }
}

// partial sums of |y - e x|^2
__global__ __launch_bounds__(256) void k_resid(const double *y, const double *x, double e, int64_t N, double *partial) {
    __shared__ double sh[8];
    double rr = 0;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < N; n += stride) {
        double r = y[n] - e * x[n];
        rr += r * r;
    }
    double tot = block_sum(rr, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// t -= sum_i c_i X_i
template <typename T>
__global__ __launch_bounds__(256) void k_subtract(const T *X, int64_t sx, int nx, const double *c, T *t, int64_t N) {
    __shared__ double cs[512];
    for (int i = threadIdx.x; i < nx; i += blockDim.x) cs[i] = c[i];
    __syncthreads();
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < N; n += stride) {
        double v = double(t[n]);
        for (int i = 0; i < nx; ++i) v -= cs[i] * double(X[i * sx + n]);
        t[n] = T(v);
    }
}

// V_j <- sum_i q[j * m + i] V_i for j < k <= KM, in place: every thread reads
// element n of all m vectors before it writes element n of the first k (U
// elements per thread, blockDim apart, for more loads in flight)
template <typename T, int KM, bool Q>
__global__ __launch_bounds__(256) void k_combine_inplace(T *V, int64_t sv, int m, const double *q, int k, int64_t N) {
    constexpr int U = Q || KM <= 8 ? 4 : 2;
    using L = Lanes<Q, U>;
    extern __shared__ double qs[];                       // [m][KM], zero beyond k
    for (int i = threadIdx.x; i < m * KM; i += blockDim.x) {
        const int row = i / KM, j = i % KM;
        qs[i] = j < k ? q[j * m + row] : 0.0;
    }
    __syncthreads();
    for (int64_t n0 = L::start(); n0 < N; n0 += L::stride()) {
        double acc[KM][U];
#pragma unroll
        for (int j = 0; j < KM; ++j)
#pragma unroll
            for (int u = 0; u < U; ++u) acc[j][u] = 0;
        for (int i = 0; i < m; ++i) {
            double v[U];
            lde<Q, U>(V + i * sv, n0, N, v);
#pragma unroll
            for (int j = 0; j < KM; ++j) {
                const double c = qs[i * KM + j];
#pragma unroll
                for (int u = 0; u < U; ++u) acc[j][u] += c * v[u];
            }
        }
#pragma unroll
        for (int j = 0; j < KM; ++j)
            if (j < k) ste<Q, U>(V + j * sv, n0, N, acc[j]);
    }
}

// (the quad form for up to 8 kept vectors: 16 of them would need 128 registers of
// accumulators for four elements)
template <typename T>
void launch_combine(T *V, int64_t sv, int m, const double *q, int k, int64_t N, int g, hipStream_t s, bool quad) {
    if (k <= 4) {
        if (quad)
            hipLaunchKernelGGL((k_combine_inplace<T, 4, true>), dim3(g), dim3(256), size_t(m) * 4 * sizeof(double), s,
                               V, sv, m, q, k, N);
        else
            hipLaunchKernelGGL((k_combine_inplace<T, 4, false>), dim3(g), dim3(256), size_t(m) * 4 * sizeof(double), s,
                               V, sv, m, q, k, N);
    } else if (k <= 8) {
        if (quad)
            hipLaunchKernelGGL((k_combine_inplace<T, 8, true>), dim3(g), dim3(256), size_t(m) * 8 * sizeof(double), s,
                               V, sv, m, q, k, N);
        else
            hipLaunchKernelGGL((k_combine_inplace<T, 8, false>), dim3(g), dim3(256), size_t(m) * 8 * sizeof(double), s,
                               V, sv, m, q, k, N);
    } else {
        hipLaunchKernelGGL((k_combine_inplace<T, kThick, false>), dim3(g), dim3(256),
                           size_t(m) * kThick * sizeof(double), s, V, sv, m, q, k, N);
    }
}

template <typename TI, typename TO>
__global__ void k_scale_copy(const TI *src, TO *dst, double f, int64_t N) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < N; n += stride) dst[n] = TO(f * double(src[n]));
}

// x[idx[i]] = v[i] and out[i] = x[idx[i]]: the P-space entries of a vector
template <typename T>
__global__ void k_put_entries(T *x, const int64_t *idx, const double *v, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[idx[i]] = T(v[i]);
}

template <typename T>
__global__ void k_get_entries(const T *x, const int64_t *idx, double *out, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = double(x[idx[i]]);
}

template <typename T>
__global__ void k_unit(T *x, int64_t N, int64_t idx) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < N; n += stride) x[n] = T(n == idx ? 1 : 0);
}

template <typename T>
__global__ void k_unit2(T *x, int64_t N, int64_t i1, int64_t i2, T v) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < N; n += stride)
        x[n] = n == i1 ? v : (n == i2 ? T(1) / T(1.4142135623730951) : T(0));
}

// Determinants a guess may use: all, or with parity p != 0 the sector
// representatives (Ia, Ib), Ia <= Ib (Ia < Ib for p = -1).  One-block spaces:
// n = I_alpha * nside + I_beta; spaces with several blocks (nside = 0): the block
// of n from the caller-layout block offsets, then the string indices.
struct SectorArgs {
    int64_t nside;
    int parity;
    const int64_t *blkoff;
    const BlockDev *blk;
    int nblk;
    const int *astart, *bstart;
};

__device__ __forceinline__ bool in_sector(const SectorArgs &a, int64_t n) {
    if (a.parity == 0) return true;
    int64_t ra, cb;
    if (a.nside > 0) {
        ra = n / a.nside;
        cb = n % a.nside;
    } else {
        int lo = 0, hi = a.nblk - 1;   // last block with blkoff <= n
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (a.blkoff[mid] <= n) lo = mid; else hi = mid - 1;
        }
        const BlockDev &B = a.blk[lo];
        const int64_t r = (n - a.blkoff[lo]) / B.nb, c = (n - a.blkoff[lo]) % B.nb;
        ra = a.astart[B.ta] + r;
        cb = a.bstart[B.tb] + c;
    }
    return !(ra > cb || (a.parity < 0 && ra == cb));
}

// out[i] = hd[i * N / ns]: an evenly spaced sample of the diagonal
__global__ void k_sample(const double *hd, int64_t N, int ns, double *out) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += gridDim.x * blockDim.x)
        out[i] = hd[int64_t(i) * N / ns];
}

// every usable n with hd[n] <= t: (hd[n], n) at the next free slot of (ov, oi)
// (cnt counts them all; at most cap are kept; the slots' order is arbitrary and the
// caller sorts them)
__global__ __launch_bounds__(256) void k_collect_below(const double *hd, int64_t N, double t, SectorArgs sa,
                                                       double *ov, int64_t *oi, unsigned long long *cnt,
                                                       int64_t cap) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < N; n += stride) {
        const double v = hd[n];
        if (!(v <= t) || !in_sector(sa, n)) continue;
        const unsigned long long pos = atomicAdd(cnt, 1ull);
        if (int64_t(pos) < cap) {
            ov[pos] = v;
            oi[pos] = n;
        }
    }
}

// lexicographic (value, index) minimum strictly above (pv, pi) over the usable
// determinants
__global__ __launch_bounds__(256) void k_argmin(const double *hd, int64_t N, double pv, int64_t pi, double *ov,
                                                int64_t *oi, SectorArgs sa) {
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    double bv = INFINITY;
    int64_t bi = -1;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < N; n += stride) {
        if (!in_sector(sa, n)) continue;
        double v = hd[n];
        bool above = (v > pv) || (v == pv && n > pi);
        if (!above) continue;
        if (v < bv || (v == bv && n < bi)) { bv = v; bi = n; }
    }
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (int(threadIdx.x) < off) {
            double v2 = sv[threadIdx.x + off];
            int64_t i2 = si[threadIdx.x + off];
            if (i2 >= 0 && (si[threadIdx.x] < 0 || v2 < sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < si[threadIdx.x]))) {
                sv[threadIdx.x] = v2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { ov[blockIdx.x] = sv[0]; oi[blockIdx.x] = si[0]; }
}


struct Dev {
    cisigma_ctx *ctx;
    hipStream_t s;
    bool quad = false;   // vector length a multiple of 4: the streaming kernels' quad form
    int ncu = 0;         // compute units of the device
    double *partial = nullptr, *dvec = nullptr, *ybuf = nullptr, *qbuf = nullptr, *pval = nullptr;
    int64_t *pidx = nullptr, *pdet = nullptr;
    int grid(int64_t N) const {
        int64_t g = (N + 255) / 256;
        return int(g < kRedBlocks ? (g > 0 ? g : 1) : kRedBlocks);
    }
};

#define DV_TRY(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            return cis_set_error(ctx, e_ == hipErrorOutOfMemory ? CISIGMA_ENOMEM : CISIGMA_EDEVICE, \
                                 std::string("davidson: ") + hipGetErrorString(e_));        \
    } while (0)

// the quad form applies when every vector starts on 16 bytes and steps by a
// multiple of 4 elements
inline bool quad_ok(const Dev &d, const void *a, int64_t sa, const void *b, int64_t sb) {
    return d.quad && (reinterpret_cast<uintptr_t>(a) & 15) == 0 && (reinterpret_cast<uintptr_t>(b) & 15) == 0 &&
           sa % 4 == 0 && sb % 4 == 0;
}

template <typename TX, typename TY>
hipError_t dots(Dev &d, const TX *X, int64_t sx, int nx, const TY *y, int64_t N, double *host_out) {
    int g = d.grid(N);
    hipLaunchKernelGGL((k_dots<TX, TY>), dim3(g), dim3(256), 0, d.s, X, sx, nx, y, N, d.partial);
    hipLaunchKernelGGL(k_reduce_partials, dim3(nx), dim3(64), 0, d.s, d.partial, g, nx, d.dvec);
    hipError_t e = hipMemcpyAsync(host_out, d.dvec, size_t(nx) * sizeof(double), hipMemcpyDeviceToHost, d.s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(d.s);
}

// out[j * nx + i] = X_i . Y_j for j < ny (blocks of kMultiY), on the host
template <typename TX, typename TY>
hipError_t dots_multi(Dev &d, const TX *X, int64_t sx, int nx, const TY *Y, int64_t sy, int ny, int64_t N,
                      double *host_out) {
    if (nx == 0 || ny == 0) return hipSuccess;
    const bool quad = quad_ok(d, X, sx, Y, sy);
    // the FP32 quad form runs at three waves per SIMD: three workgroups per
    // compute unit, so that the whole grid is resident at once
    int g = d.grid(N);
    if (quad && sizeof(TX) == 4 && d.ncu > 0) g = std::min(g, 3 * d.ncu);
    for (int j0 = 0; j0 < ny; j0 += kMultiY) {
        const int nyc = std::min(kMultiY, ny - j0);
        if (quad)
            hipLaunchKernelGGL((k_dots_multi<TX, TY, true>), dim3(g), dim3(256), 0, d.s, X, sx, nx,
                               Y + int64_t(j0) * sy, sy, nyc, N, d.partial);
        else
            hipLaunchKernelGGL((k_dots_multi<TX, TY, false>), dim3(g), dim3(256), 0, d.s, X, sx, nx,
                               Y + int64_t(j0) * sy, sy, nyc, N, d.partial);
        hipLaunchKernelGGL(k_reduce_partials, dim3(nx * nyc), dim3(64), 0, d.s, d.partial, g, nx * nyc,
                           d.dvec);
        hipError_t e = hipMemcpyAsync(host_out + size_t(j0) * nx, d.dvec, size_t(nx) * nyc * sizeof(double),
                                      hipMemcpyDeviceToHost, d.s);
        if (e != hipSuccess) return e;
    }
    return hipStreamSynchronize(d.s);
}

// T_j -= sum_i c[j * nx + i] X_i for j < ny (host coefficients)
template <typename T>
hipError_t subtract_multi(Dev &d, const T *X, int64_t sx, int nx, const double *host_c, int ny, T *Tv, int64_t st,
                          int64_t N) {
    if (nx == 0 || ny == 0) return hipSuccess;
    const int g = d.grid(N);
    for (int j0 = 0; j0 < ny; j0 += kMultiY) {
        const int nyc = std::min(kMultiY, ny - j0);
        hipError_t e = hipMemcpyAsync(d.dvec, host_c + size_t(j0) * nx, size_t(nx) * nyc * sizeof(double),
                                      hipMemcpyHostToDevice, d.s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_subtract_multi<T>), dim3(g), dim3(256), 0, d.s, X, sx, nx, d.dvec, nyc,
                           Tv + int64_t(j0) * st, st, N);
    }
    return hipGetLastError();
}

// T_j -= sum_i c[j * nx + i] X_i for j < ny <= kMultiY; returns on the host the
// squared norms before the update (pre[j]) and the Gram matrix of the results
// (gram[j * ny + k], both triangles)
template <typename T>
hipError_t subtract_gram(Dev &d, const T *X, int64_t sx, int nx, const double *host_c, int ny, T *Tv, int64_t st,
                         int64_t N, double *pre, double *gram) {
    const int g = d.grid(N);
    const int nv = ny + ny * (ny + 1) / 2;
    hipError_t e = hipSuccess;
    if (nx > 0) e = hipMemcpyAsync(d.dvec, host_c, size_t(nx) * ny * sizeof(double), hipMemcpyHostToDevice, d.s);
    if (e != hipSuccess) return e;
#define CIS_SUBG(NY, Q)                                                                                     \
    hipLaunchKernelGGL((k_subtract_gram<T, NY, Q>), dim3(g), dim3(256), 0, d.s, X, sx, nx, d.dvec, Tv, st, N, \
                       d.partial)
    // (quad form up to three corrections: four need 158 registers, fewer than four
    // waves per SIMD)
    const bool quad = ny <= 3 && quad_ok(d, X, sx, Tv, st);
    switch (ny * 2 + (quad ? 1 : 0)) {
        case 2: CIS_SUBG(1, false); break;
        case 3: CIS_SUBG(1, true); break;
        case 4: CIS_SUBG(2, false); break;
        case 5: CIS_SUBG(2, true); break;
        case 6: CIS_SUBG(3, false); break;
        case 7: CIS_SUBG(3, true); break;
        case 8: CIS_SUBG(4, false); break;
        default: return hipErrorInvalidValue;
    }
#undef CIS_SUBG
    hipLaunchKernelGGL(k_reduce_partials, dim3(nv), dim3(64), 0, d.s, d.partial, g, nv, d.dvec);
    std::vector<double> out(nv);
    e = hipMemcpyAsync(out.data(), d.dvec, size_t(nv) * sizeof(double), hipMemcpyDeviceToHost, d.s);
    if (e == hipSuccess) e = hipStreamSynchronize(d.s);
    if (e != hipSuccess) return e;
    int q = ny;
    for (int j = 0; j < ny; ++j) {
        pre[j] = out[j];
        for (int k = 0; k <= j; ++k, ++q) gram[size_t(j) * ny + k] = gram[size_t(k) * ny + j] = out[q];
    }
    return hipSuccess;
}

// D_j = sum_k w[j * ny + k] T_k for j < nd, ny <= kMultiY (host coefficients)
template <typename T>
hipError_t combine_new(Dev &d, const T *Tv, int64_t st, int ny, const double *host_w, int nd, T *D, int64_t sd,
                       int64_t N) {
    if (nd == 0) return hipSuccess;
    const int g = d.grid(N);
    hipError_t e = hipMemcpyAsync(d.dvec, host_w, size_t(nd) * ny * sizeof(double), hipMemcpyHostToDevice, d.s);
    if (e != hipSuccess) return e;
#define CIS_COMB(NY, Q) \
    hipLaunchKernelGGL((k_combine_new<T, NY, Q>), dim3(g), dim3(256), 0, d.s, Tv, st, d.dvec, nd, D, sd, N)
    const bool quad = quad_ok(d, Tv, st, D, sd);
    switch (ny * 2 + (quad ? 1 : 0)) {
        case 2: CIS_COMB(1, false); break;
        case 3: CIS_COMB(1, true); break;
        case 4: CIS_COMB(2, false); break;
        case 5: CIS_COMB(2, true); break;
        case 6: CIS_COMB(3, false); break;
        case 7: CIS_COMB(3, true); break;
        case 8: CIS_COMB(4, false); break;
        case 9: CIS_COMB(4, true); break;
        default: return hipErrorInvalidValue;
    }
#undef CIS_COMB
    return hipGetLastError();
}

template <typename T>
int run(cisigma_ctx *ctx, int nroots, double tol, double *energies, void *vecs, cisigma_stats *stats) {
    auto t0 = std::chrono::steady_clock::now();
    const bool mixed = std::is_same<T, float>::value;
    const int dt = mixed ? CISIGMA_FP32 : CISIGMA_FP64;
    const int64_t N = ctx->lay.ndet;
    const size_t es = sizeof(T);
    // sigma workspaces left by earlier apply calls (their materialised same-spin
    // rows take half of what was free) are released when the basis would not fit
    // beside them at full size; the next sigma allocates them again, sized to
    // what is free then
    {
        const int want = ctx->max_space > 0 ? ctx->max_space : std::max(8 * nroots, 32);
        const size_t need = size_t(2 * want + 2 * nroots) * N * es + size_t(nroots + 1) * N * 8 +
                            (mixed ? size_t(N) * 8 : 0);
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess && need + (256u << 20) > size_t(0.7 * double(fr))) {
            int rc0 = release_workspace(ctx, CISIGMA_FP32);
            if (rc0 == CISIGMA_OK) rc0 = release_workspace(ctx, CISIGMA_FP64);
            if (rc0) return rc0;
        }
    }
    int max_space = ctx->max_space;
    if (max_space <= 0) {
        // default: a generous subspace (restarts slow Davidson down on strongly
        // correlated spaces), capped by what fits in 70% of free device memory
        max_space = std::max(8 * nroots, 32);
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
            size_t fixed = size_t(2 * nroots) * N * es + size_t(nroots + 1) * N * 8 + (mixed ? size_t(N) * 8 : 0);
            size_t avail = size_t(0.7 * double(fr));
            int fit = avail > fixed ? int((avail - fixed) / (2 * size_t(N) * es)) : 0;
            max_space = std::min(max_space, fit);
        }
    }
    max_space = std::max(max_space, 2 * nroots);
    // M_S = 0 sector (Sec. 3.1, Sec. 3.3): vectors with C(Ib, Ia) = par C(Ia, Ib)
    const int par = ctx->spin_parity;
    // one-block spaces index the sector by n = I_alpha * nside + I_beta; with
    // several (mirror) blocks nside = 0 and the blocks are decoded
    const int64_t nside = par && ctx->cas ? int64_t(ctx->sp[0].nstr) : 0;
    int64_t dim = N;
    if (par && ctx->cas) {
        dim = par > 0 ? nside * (nside + 1) / 2 : nside * (nside - 1) / 2;
    } else if (par) {
        dim = 0;   // pairs I_alpha <= I_beta (< for p = -1) over the blocks
        for (int b = 0; b < ctx->lay.nblk; ++b) {
            const int ta = ctx->lay.blk_a[b], tb = ctx->lay.blk_b[b];
            const int64_t na = ctx->sp[0].tcount[ta], nb = ctx->sp[1].tcount[tb];
            if (ta < tb) dim += na * nb;
            else if (ta == tb) dim += par > 0 ? na * (na + 1) / 2 : na * (na - 1) / 2;
        }
    }
    if (nroots > dim)
        return cis_set_error(ctx, CISIGMA_EINVAL, "davidson: nroots exceeds the dimension of the spin-parity sector");
    if (int64_t(max_space) > dim) max_space = int(dim);
    if (max_space > 512) max_space = 512;
    double rtol = ctx->resid_tol > 0 ? ctx->resid_tol : std::sqrt(tol);
    if (mixed && ctx->resid_tol <= 0) rtol = std::max(rtol, 1e-5);
    Dev d{ctx, ctx->stream};
    d.quad = N % 4 == 0;   // every vector below is its own allocation with stride N
    if (hipDeviceGetAttribute(&d.ncu, hipDeviceAttributeMultiprocessorCount, ctx->dev) != hipSuccess) d.ncu = 0;
    T *B = nullptr, *S = nullptr, *SX = nullptr, *TB = nullptr;
    double *X64 = nullptr, *hd = nullptr, *sig64 = nullptr;
    // free-memory check before the big allocations
    {
        size_t need = size_t(2 * max_space + 2 * nroots) * N * es + size_t(nroots + 1) * N * 8 +
                      (mixed ? size_t(N) * 8 : 0);
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess && need + (256u << 20) > fr)
            return cis_set_error(ctx, CISIGMA_ENOMEM, "davidson: not enough device memory for the subspace");
    }
    auto cleanup = [&]() {
        (void)hipFree(B); (void)hipFree(S); (void)hipFree(SX); (void)hipFree(TB); (void)hipFree(X64);
        (void)hipFree(hd); (void)hipFree(sig64);
        (void)hipFree(d.partial); (void)hipFree(d.dvec); (void)hipFree(d.pidx); (void)hipFree(d.ybuf);
        (void)hipFree(d.qbuf); (void)hipFree(d.pval); (void)hipFree(d.pdet);
    };
    struct Guard { std::function<void()> f; ~Guard() { f(); } } guard{cleanup};
    DV_TRY(hipMalloc(&B, size_t(max_space) * N * es));
    DV_TRY(hipMalloc(&S, size_t(max_space) * N * es));
    DV_TRY(hipMalloc(&SX, size_t(nroots) * N * es));
    DV_TRY(hipMalloc(&TB, size_t(nroots) * N * es));
    DV_TRY(hipMalloc(&X64, size_t(nroots) * N * 8));
    DV_TRY(hipMalloc(&hd, size_t(N) * 8));
    if (mixed) DV_TRY(hipMalloc(&sig64, size_t(N) * 8));
    DV_TRY(hipMalloc(&d.partial, size_t(kRedBlocks) * 512 * kMultiY * sizeof(double)));
    // per-block (argmin) or per-vector (dots: <= 512 x kMultiY) results and coefficients
    DV_TRY(hipMalloc(&d.dvec, size_t(std::max(kRedBlocks, 512 * kMultiY)) * sizeof(double)));
    DV_TRY(hipMalloc(&d.pidx, kRedBlocks * sizeof(int64_t)));
    DV_TRY(hipMalloc(&d.ybuf, size_t(kRitzRoots) * (512 + 1) * sizeof(double)));
    DV_TRY(hipMalloc(&d.qbuf, size_t(kThick) * 512 * sizeof(double)));
    DV_TRY(launch_hdiag(ctx, hd, d.s));

    const int g = d.grid(N);
    auto symmetrize = [&](T *t) -> hipError_t {
        return ctx->cas ? launch_symmetrize(t, int(nside), par, dt, d.s) : launch_symmetrize_blocks(ctx, t, par, dt, d.s);
    };
    // P-space: the np determinants with the lowest H_II (ties: lowest index) and
    // the exact H over them, diagonalised: its lowest eigenvectors are the guess,
    // and on those determinants the correction is (theta - H_PP)^-1 r_P
    const int np = (par == 0 && ctx->pspace >= nroots) ? int(std::min<int64_t>(ctx->pspace, dim)) : 0;
    std::vector<int64_t> pdet;
    std::vector<double> pdiag, pw, pU;
    // (1) guess: unit vectors on the lowest diagonal elements (ties: lowest index),
    // or the lowest eigenvectors of the P-space block
    {
        double pv = -INFINITY;
        int64_t pi = -1;
        std::vector<uint32_t> sa, sb;   // strings, for the mirror determinants of sector guesses
        const int nlow = std::max(nroots, np);
        const SectorArgs sec{nside, par, ctx->d_blkoff, ctx->bt.blk, ctx->lay.nblk, ctx->d_tstart[0],
                             ctx->d_tstart[1]};
        // the nlow usable determinants of lowest (H_II, index), in that order: every
        // one with H_II <= t is collected for a threshold t from an evenly spaced
        // sample of H_II, raised until at least nlow are, and sorted here (then the
        // first nlow are exactly the lowest); one argmin pass per determinant when
        // more than the collection buffer tie at the threshold
        std::vector<std::pair<double, int64_t>> low;
        {
            const int ns = int(std::min<int64_t>(N, 16384));
            std::vector<double> samp(ns);
            hipLaunchKernelGGL(k_sample, dim3((ns + 255) / 256), dim3(256), 0, d.s, hd, N, ns, d.partial);
            DV_TRY(hipMemcpyAsync(samp.data(), d.partial, ns * sizeof(double), hipMemcpyDeviceToHost, d.s));
            DV_TRY(hipStreamSynchronize(d.s));
            std::sort(samp.begin(), samp.end());
            // collection buffer: the first cap doubles of d.partial and the cap after them
            const int64_t cap = int64_t(1) << 18;
            static_assert((int64_t(1) << 19) <= int64_t(kRedBlocks) * 512 * kMultiY, "collection buffer");
            double *cv = d.partial;
            int64_t *ci = reinterpret_cast<int64_t *>(d.partial + cap);
            auto *cnt = reinterpret_cast<unsigned long long *>(d.pidx);
            int64_t k = std::max<int64_t>(1, (int64_t(nlow) * ns + N - 1) / N) + 1;   // sample rank of t
            while (true) {
                const double t = k > ns ? INFINITY : samp[size_t(k - 1)];
                const unsigned long long zero = 0;
                unsigned long long c = 0;
                DV_TRY(hipMemcpyAsync(cnt, &zero, sizeof(zero), hipMemcpyHostToDevice, d.s));
                hipLaunchKernelGGL(k_collect_below, dim3(g), dim3(256), 0, d.s, hd, N, t, sec, cv, ci, cnt, cap);
                DV_TRY(hipMemcpyAsync(&c, cnt, sizeof(c), hipMemcpyDeviceToHost, d.s));
                DV_TRY(hipStreamSynchronize(d.s));
                if (int64_t(c) > cap) break;   // ties beyond the buffer: the argmin passes below
                if (int64_t(c) >= nlow || k > ns) {
                    std::vector<double> v(c);
                    std::vector<int64_t> ix(c);
                    if (c > 0) {
                        DV_TRY(hipMemcpyAsync(v.data(), cv, c * sizeof(double), hipMemcpyDeviceToHost, d.s));
                        DV_TRY(hipMemcpyAsync(ix.data(), ci, c * sizeof(int64_t), hipMemcpyDeviceToHost, d.s));
                        DV_TRY(hipStreamSynchronize(d.s));
                    }
                    for (size_t i = 0; i < size_t(c); ++i) low.emplace_back(v[i], ix[i]);
                    std::sort(low.begin(), low.end());
                    if (low.size() > size_t(nlow)) low.resize(nlow);
                    break;
                }
                k *= 4;
            }
        }
        if (low.empty()) {
            std::vector<double> hv(g);
            std::vector<int64_t> hi(g);
            for (int r = 0; r < nlow; ++r) {
                hipLaunchKernelGGL(k_argmin, dim3(g), dim3(256), 0, d.s, hd, N, pv, pi, d.dvec, d.pidx, sec);
                DV_TRY(hipMemcpyAsync(hv.data(), d.dvec, g * sizeof(double), hipMemcpyDeviceToHost, d.s));
                DV_TRY(hipMemcpyAsync(hi.data(), d.pidx, g * sizeof(int64_t), hipMemcpyDeviceToHost, d.s));
                DV_TRY(hipStreamSynchronize(d.s));
                double bv = INFINITY;
                int64_t bi = -1;
                for (int b = 0; b < g; ++b)
                    if (hi[b] >= 0 && (bi < 0 || hv[b] < bv || (hv[b] == bv && hi[b] < bi))) { bv = hv[b]; bi = hi[b]; }
                if (bi < 0) break;
                pv = bv;
                pi = bi;
                low.emplace_back(bv, bi);
            }
        }
        if (low.size() < size_t(nlow)) return cis_set_error(ctx, CISIGMA_EINVAL, "davidson: fewer determinants than roots");
        for (int r = 0; r < nlow; ++r) {
            const double bv = low[size_t(r)].first;
            const int64_t bi = low[size_t(r)].second;
            if (np > 0) {
                pdet.push_back(bi);
                pdiag.push_back(bv);
                continue;
            }
            int64_t mirror = bi;   // the determinant with the strings exchanged
            if (par && ctx->cas) {
                mirror = (bi % nside) * nside + bi / nside;
            } else if (par) {
                if (sa.empty()) {
                    sa.resize(ctx->sp[0].nstr);
                    sb.resize(ctx->sp[1].nstr);
                    DV_TRY(hipMemcpy(sa.data(), ctx->sp[0].d_str, sa.size() * 4, hipMemcpyDeviceToHost));
                    DV_TRY(hipMemcpy(sb.data(), ctx->sp[1].d_str, sb.size() * 4, hipMemcpyDeviceToHost));
                }
                uint32_t xa = 0, xb = 0;
                if (!det_strings(ctx, bi, sa, sb, &xa, &xb) || cisigma_address(ctx, xb, xa, &mirror) != CISIGMA_OK ||
                    mirror < 0)
                    return cis_set_error(ctx, CISIGMA_EINVAL, "davidson: guess outside the spin-parity sector");
            }
            if (par == 0 || mirror == bi)
                hipLaunchKernelGGL(k_unit<T>, dim3(g), dim3(256), 0, d.s, B + int64_t(r) * N, N, bi);
            else   // (|Ia Ib> + p |Ib Ia>) / sqrt(2)
                hipLaunchKernelGGL(k_unit2<T>, dim3(g), dim3(256), 0, d.s, B + int64_t(r) * N, N, mirror, bi,
                                   T(par) / T(1.4142135623730951));
        }
        if (np > 0) {
            std::vector<uint32_t> astr(ctx->sp[0].nstr), bstr(ctx->sp[1].nstr), pa(np), pb(np);
            if (!astr.empty())
                DV_TRY(hipMemcpy(astr.data(), ctx->sp[0].d_str, astr.size() * 4, hipMemcpyDeviceToHost));
            if (!bstr.empty())
                DV_TRY(hipMemcpy(bstr.data(), ctx->sp[1].d_str, bstr.size() * 4, hipMemcpyDeviceToHost));
            for (int i = 0; i < np; ++i)
                if (!det_strings(ctx, pdet[i], astr, bstr, &pa[i], &pb[i]))
                    return cis_set_error(ctx, CISIGMA_EINVAL, "davidson: P-space index outside the space");
            std::vector<double> hpp(size_t(np) * np);
            for (int i = 0; i < np; ++i)
                for (int j = 0; j <= i; ++j)
                    hpp[size_t(i) * np + j] = hpp[size_t(j) * np + i] = hmat_element(ctx, pa[i], pb[i], pa[j], pb[j]);
            sym_eig(hpp, np, pw, pU);
            DV_TRY(hipMalloc(&d.pdet, size_t(np) * sizeof(int64_t)));
            DV_TRY(hipMalloc(&d.pval, size_t(np) * nroots * sizeof(double)));
            DV_TRY(hipMemcpy(d.pdet, pdet.data(), size_t(np) * sizeof(int64_t), hipMemcpyHostToDevice));
            std::vector<double> u(size_t(np) * nroots);
            for (int r = 0; r < nroots; ++r)
                for (int i = 0; i < np; ++i) u[size_t(r) * np + i] = pU[size_t(i) * np + r];
            DV_TRY(hipMemcpy(d.pval, u.data(), u.size() * sizeof(double), hipMemcpyHostToDevice));
            const int pg = std::min(64, (np + 255) / 256);
            for (int r = 0; r < nroots; ++r) {
                hipLaunchKernelGGL(k_unit<T>, dim3(g), dim3(256), 0, d.s, B + int64_t(r) * N, N, int64_t(-1));
                hipLaunchKernelGGL(k_put_entries<T>, dim3(pg), dim3(256), 0, d.s, B + int64_t(r) * N, d.pdet,
                                   d.pval + size_t(r) * np, np);
            }
            DV_TRY(hipGetLastError());
        }
    }
    // corrections on the P-space determinants of every root: TB holds
    // t = r / (theta - H_II) there; r_P is recovered and solved exactly
    auto pspace_correct = [&](const std::vector<double> &theta) -> hipError_t {
        if (np == 0) return hipSuccess;
        const int pg = std::min(64, (np + 255) / 256);
        for (int r = 0; r < nroots; ++r)
            hipLaunchKernelGGL(k_get_entries<T>, dim3(pg), dim3(256), 0, d.s, TB + int64_t(r) * N, d.pdet,
                               d.pval + size_t(r) * np, np);
        std::vector<double> t(size_t(np) * nroots), y(np);
        hipError_t e = hipMemcpyAsync(t.data(), d.pval, t.size() * sizeof(double), hipMemcpyDeviceToHost, d.s);
        if (e == hipSuccess) e = hipStreamSynchronize(d.s);
        if (e != hipSuccess) return e;
        auto clamp = [](double x) { return std::fabs(x) < 1e-8 ? (x < 0 ? -1e-8 : 1e-8) : x; };
        for (int r = 0; r < nroots; ++r) {
            double *tr = t.data() + size_t(r) * np;
            for (int i = 0; i < np; ++i) tr[i] *= clamp(theta[r] - pdiag[i]);          // r_P
            for (int k = 0; k < np; ++k) {
                double acc = 0;
                for (int i = 0; i < np; ++i) acc += pU[size_t(i) * np + k] * tr[i];
                y[k] = acc / clamp(theta[r] - pw[k]);
            }
            for (int i = 0; i < np; ++i) {
                double acc = 0;
                for (int k = 0; k < np; ++k) acc += pU[size_t(i) * np + k] * y[k];
                tr[i] = acc;
            }
        }
        e = hipMemcpyAsync(d.pval, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, d.s);
        if (e != hipSuccess) return e;
        for (int r = 0; r < nroots; ++r)
            hipLaunchKernelGGL(k_put_entries<T>, dim3(pg), dim3(256), 0, d.s, TB + int64_t(r) * N, d.pdet,
                               d.pval + size_t(r) * np, np);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(d.s);   // t is host memory
        return e;
    };
    std::vector<double> G(size_t(max_space) * max_space, 0.0);
    std::vector<double> theta(nroots, 0.0), theta_old(nroots, INFINITY), rnorm(nroots, 0.0);
    std::vector<double> erq(nroots, 0.0), r64(nroots, INFINITY);
    std::vector<double> w, Y, col(max_space + 8);
    int m = 0, nnew = nroots, iter = 0, nsig32 = 0, nsig64 = 0, nref = 0;
    // JSON-lines log (cisigma_set_log): one line per iteration and per FP64 refinement
    FILE *logf = ctx->log_path.empty() ? nullptr : std::fopen(ctx->log_path.c_str(), "a");
    const int call = ++ctx->log_calls;
    struct LogClose { FILE *f; ~LogClose() { if (f) std::fclose(f); } } log_close{logf};
    auto secs = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    auto log_line = [&](const char *kind, int k, const double *e, const double *res) {
        if (!logf) return;
        std::fprintf(logf, "{\"call\": %d, \"%s\": %d, \"dim\": %d, \"precision\": \"%s\", \"energies\": [", call,
                     kind, k, m, mixed ? "mixed" : "fp64");
        for (int r = 0; r < nroots; ++r) std::fprintf(logf, "%s%.15g", r ? ", " : "", e[r]);
        std::fprintf(logf, "], \"residuals\": [");
        for (int r = 0; r < nroots; ++r) std::fprintf(logf, "%s%.6g", r ? ", " : "", res[r]);
        std::fprintf(logf, "], \"sigma_fp32\": %d, \"sigma_fp64\": %d, \"seconds\": %.6f}\n", nsig32, nsig64, secs());
        std::fflush(logf);
    };
    bool converged = false, have_rq = false, stalled = false;
    int since_ref = 0;
    int rc = CISIGMA_OK;
    // Ritz coefficients of the previous iteration (mprev x nroots) in the current
    // basis, whose first mprev vectors are unchanged since: a thick restart keeps
    // the part of them outside the current Ritz vectors
    const bool thick = ctx->thick_restart && 3 * nroots <= max_space && 2 * nroots <= kThick;
    std::vector<double> Yprev;
    int mprev = 0;
    bool prev_ok = false;
    auto sigma_of = [&](const void *x, void *y, int dtype) -> int {
        int r = apply_sigma(ctx, x, y, dtype, d.s);
        if (dtype == CISIGMA_FP32) ++nsig32; else ++nsig64;
        return r;
    };
    // Ritz vectors (FP64) and their sigma (when want_x: they are read only by the
    // FP64 refinement, a plain collapse and the output), and the corrections, for
    // all roots from the eigenvectors Yv (m x m, column r = root r); optionally the
    // residual norms.  x_fresh: X64 and SX hold the Ritz vectors of the basis as it is.
    bool x_fresh = false;
    auto ritz_all = [&](int mm, const std::vector<double> &Yv, bool norms, bool want_x) -> hipError_t {
        x_fresh = want_x;
        for (int r0 = 0; r0 < nroots; r0 += kRitzRoots) {
            const int nr = std::min(kRitzRoots, nroots - r0);
            std::vector<double> yy(size_t(nr) * mm + nr);
            for (int r = 0; r < nr; ++r)
                for (int i = 0; i < mm; ++i) yy[size_t(r) * mm + i] = Yv[size_t(i) * mm + r0 + r];
            for (int r = 0; r < nr; ++r) yy[size_t(nr) * mm + r] = theta[r0 + r];
            hipError_t e = hipMemcpyAsync(d.ybuf, yy.data(), yy.size() * sizeof(double), hipMemcpyHostToDevice, d.s);
            if (e != hipSuccess) return e;
#define CIS_RITZ1(RR, WXX, QQ)                                                                                  \
    hipLaunchKernelGGL((k_ritz_multi<T, RR, WXX, QQ>), dim3(g), dim3(256), 0, d.s, B, S, N, mm, nr, d.ybuf,         \
                       d.ybuf + size_t(nr) * mm, hd, X64 + int64_t(r0) * N, SX + int64_t(r0) * N,                 \
                       TB + int64_t(r0) * N, N, d.partial)
#define CIS_RITZ(RR, WXX)              \
    do {                               \
        if (d.quad)                    \
            CIS_RITZ1(RR, WXX, true);  \
        else                           \
            CIS_RITZ1(RR, WXX, false); \
    } while (0)
            static_assert(kRitzRoots == 4, "one instantiation per root count");
            switch (nr * 2 + (want_x ? 1 : 0)) {
                case 2: CIS_RITZ(1, false); break;
                case 3: CIS_RITZ(1, true); break;
                case 4: CIS_RITZ(2, false); break;
                case 5: CIS_RITZ(2, true); break;
                case 6: CIS_RITZ(3, false); break;
                case 7: CIS_RITZ(3, true); break;
                case 8: CIS_RITZ(4, false); break;
                default: CIS_RITZ(4, true); break;
            }
#undef CIS_RITZ
#undef CIS_RITZ1
            if (norms) {
                std::vector<double> part(size_t(nr) * g);
                e = hipMemcpyAsync(part.data(), d.partial, part.size() * sizeof(double), hipMemcpyDeviceToHost, d.s);
                if (e == hipSuccess) e = hipStreamSynchronize(d.s);
                if (e != hipSuccess) return e;
                for (int r = 0; r < nr; ++r) {
                    double ss = 0;
                    for (int b = 0; b < g; ++b) ss += part[size_t(r) * g + b];
                    rnorm[r0 + r] = std::sqrt(ss);
                }
            }
        }
        return hipGetLastError();
    };
    while (true) {
        // (4) sigma of the new vectors and the new columns of G (one pass over the
        // basis for all new columns)
        for (int k = m; k < m + nnew; ++k) {
            rc = sigma_of(B + int64_t(k) * N, S + int64_t(k) * N, dt);
            if (rc) return rc;
        }
        if (nnew > 0) {
            std::vector<double> gc(size_t(m + nnew) * nnew);
            DV_TRY(dots_multi(d, B, N, m + nnew, S + int64_t(m) * N, N, nnew, N, gc.data()));
            for (int j = 0; j < nnew; ++j) {
                const int k = m + j;
                for (int i = 0; i <= k; ++i)
                    G[size_t(i) * max_space + k] = G[size_t(k) * max_space + i] = gc[size_t(j) * (m + nnew) + i];
            }
        }
        m += nnew;
        std::vector<double> Gm(size_t(m) * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j)
                Gm[size_t(i) * m + j] = 0.5 * (G[size_t(i) * max_space + j] + G[size_t(j) * max_space + i]);
        sym_eig(Gm, m, w, Y);
        ++iter;
        ++since_ref;
        for (int r = 0; r < nroots; ++r) theta[r] = w[r];
        // residual norms and corrections (the Ritz vectors themselves when needed below)
        DV_TRY(ritz_all(m, Y, true, false));
        bool all_ok = true;
        for (int r = 0; r < nroots; ++r)
            if (!(std::fabs(theta[r] - theta_old[r]) <= tol && rnorm[r] <= rtol)) all_ok = false;
        log_line("iteration", iter, theta.data(), rnorm.data());
        if (ctx->verbose) {
            std::fprintf(stderr, "davidson it %3d dim %3d", iter, m);
            for (int r = 0; r < nroots; ++r) std::fprintf(stderr, "  E%d %.12f |r| %.3e", r, theta[r], rnorm[r]);
            std::fprintf(stderr, "\n");
        }
        for (int r = 0; r < nroots; ++r) theta_old[r] = theta[r];
        bool refined_now = false;
        if (mixed && (all_ok || (ctx->refine_every > 0 && since_ref >= ctx->refine_every) || iter >= ctx->max_iter)) {
            // FP64 refinement: rebuild sigma of the Ritz vectors in FP64
            if (!x_fresh) DV_TRY(ritz_all(m, Y, false, true));
            refined_now = true;
            ++nref;
            since_ref = 0;
            bool ok64 = true;
            // spaces where both precisions' sigma workspaces do not fit beside the
            // basis (CAS(18,18) with FP32 vectors): the FP32 one makes room for the
            // FP64 one during the refinement
            const bool swap = ctx->low_memory || !workspace_fits(ctx, CISIGMA_FP64);
            if (swap) {
                rc = release_workspace(ctx, CISIGMA_FP32);
                if (rc) return rc;
            }
            for (int r = 0; r < nroots; ++r) {
                double *x = X64 + int64_t(r) * N;
                rc = sigma_of(x, sig64, CISIGMA_FP64);
                if (rc) return rc;
                double xs, xx;
                DV_TRY(dots(d, x, N, 1, sig64, N, &xs));
                DV_TRY(dots(d, x, N, 1, x, N, &xx));
                erq[r] = xs / xx;
                // residual of the FP64 Ritz vector: |sigma - E x| / |x|
                hipLaunchKernelGGL(k_resid, dim3(g), dim3(256), 0, d.s, sig64, x, erq[r], N, d.partial);
                std::vector<double> part(g);
                DV_TRY(hipMemcpyAsync(part.data(), d.partial, g * sizeof(double), hipMemcpyDeviceToHost, d.s));
                DV_TRY(hipStreamSynchronize(d.s));
                double r2 = 0;
                for (double v : part) r2 += v;
                r64[r] = std::sqrt(r2 / xx);
                if (r64[r] > rtol) ok64 = false;
                // collapse slot r: basis = x (FP32), sigma = FP64 sigma rounded
                hipLaunchKernelGGL((k_scale_copy<double, T>), dim3(g), dim3(256), 0, d.s, x, TB + int64_t(r) * N,
                                   1.0, N);
                hipLaunchKernelGGL((k_scale_copy<double, T>), dim3(g), dim3(256), 0, d.s, sig64, SX + int64_t(r) * N,
                                   1.0, N);
            }
            if (swap) {
                rc = release_workspace(ctx, CISIGMA_FP64);
                if (rc) return rc;
            }
            have_rq = true;
            log_line("refinement", nref, erq.data(), r64.data());
            if (ctx->verbose) {
                std::fprintf(stderr, "  refine %d:", nref);
                for (int r = 0; r < nroots; ++r) std::fprintf(stderr, "  E%d %.12f |r64| %.3e", r, erq[r], r64[r]);
                std::fprintf(stderr, "\n");
            }
            if (ok64) { converged = true; break; }
            // restart from the collapsed FP64-refined Ritz vectors
            for (int r = 0; r < nroots; ++r) {
                DV_TRY(hipMemcpyAsync(B + int64_t(r) * N, TB + int64_t(r) * N, N * es, hipMemcpyDeviceToDevice, d.s));
                DV_TRY(hipMemcpyAsync(S + int64_t(r) * N, SX + int64_t(r) * N, N * es, hipMemcpyDeviceToDevice, d.s));
            }
            // exact projected matrix of the collapsed basis
            for (int k = 0; k < nroots; ++k) {
                DV_TRY(dots(d, B, N, nroots, S + int64_t(k) * N, N, col.data()));
                for (int i = 0; i < nroots; ++i) G[size_t(i) * max_space + k] = col[i];
            }
            for (int i = 0; i < nroots; ++i)
                for (int k = 0; k < i; ++k)
                    G[size_t(i) * max_space + k] = G[size_t(k) * max_space + i] =
                        0.5 * (G[size_t(i) * max_space + k] + G[size_t(k) * max_space + i]);
            m = nroots;
            if (iter >= ctx->max_iter) break;
            // corrections from the refined residuals: recompute Ritz pieces in the collapsed basis
            std::vector<double> Gm2(size_t(m) * m);
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j) Gm2[size_t(i) * m + j] = G[size_t(i) * max_space + j];
            sym_eig(Gm2, m, w, Y);
            for (int r = 0; r < nroots; ++r) theta[r] = w[r];
            DV_TRY(ritz_all(m, Y, false, true));
        } else if (!mixed) {
            if (all_ok) { converged = true; break; }
        }
        if (iter >= ctx->max_iter) break;
        bool collapsed = refined_now;
        // a collapse changes the basis: the Ritz vectors of this iteration are kept
        // first (the plain collapse reads them, and a later exit returns them)
        if (!refined_now && m + nroots > max_space && !x_fresh) DV_TRY(ritz_all(m, Y, false, true));
        if (!refined_now && m + nroots > max_space && thick && prev_ok && mprev <= m) {
            // thick restart: the current Ritz vectors plus the orthonormalised
            // remainder of the previous ones, B <- B Q and S <- S Q in place,
            // G <- Q^T G Q
            std::vector<double> Q(size_t(2 * nroots) * m, 0.0);
            for (int r = 0; r < nroots; ++r)
                for (int i = 0; i < m; ++i) Q[size_t(r) * m + i] = Y[size_t(i) * m + r];
            int k = nroots;
            std::vector<double> v(m);
            for (int r = 0; r < nroots; ++r) {
                double n0 = 0;
                for (int i = 0; i < m; ++i) {
                    v[i] = i < mprev ? Yprev[size_t(i) * nroots + r] : 0.0;
                    n0 += v[i] * v[i];
                }
                for (int pass = 0; pass < 2; ++pass)
                    for (int j = 0; j < k; ++j) {
                        double c = 0;
                        for (int i = 0; i < m; ++i) c += Q[size_t(j) * m + i] * v[i];
                        for (int i = 0; i < m; ++i) v[i] -= c * Q[size_t(j) * m + i];
                    }
                double nv = 0;
                for (int i = 0; i < m; ++i) nv += v[i] * v[i];
                if (!(nv > 1e-8 * n0)) continue;
                nv = std::sqrt(nv);
                for (int i = 0; i < m; ++i) Q[size_t(k) * m + i] = v[i] / nv;
                ++k;
            }
            if (k > nroots) {
                DV_TRY(hipMemcpyAsync(d.qbuf, Q.data(), size_t(k) * m * sizeof(double), hipMemcpyHostToDevice, d.s));
                launch_combine<T>(B, N, m, d.qbuf, k, N, g, d.s, d.quad);
                launch_combine<T>(S, N, m, d.qbuf, k, N, g, d.s, d.quad);
                DV_TRY(hipGetLastError());
                std::vector<double> GQ(size_t(m) * k, 0.0);
                for (int i = 0; i < m; ++i)
                    for (int b = 0; b < k; ++b) {
                        double acc = 0;
                        for (int l = 0; l < m; ++l) acc += Gm[size_t(i) * m + l] * Q[size_t(b) * m + l];
                        GQ[size_t(i) * k + b] = acc;
                    }
                for (int i = 0; i < max_space * max_space; ++i) G[i] = 0;
                for (int a = 0; a < k; ++a)
                    for (int b = 0; b <= a; ++b) {
                        double acc = 0;
                        for (int i = 0; i < m; ++i) acc += Q[size_t(a) * m + i] * GQ[size_t(i) * k + b];
                        G[size_t(a) * max_space + b] = G[size_t(b) * max_space + a] = acc;
                    }
                m = k;
                collapsed = true;
            }
        }
        if (!collapsed && m + nroots > max_space) {
            // collapse onto the current Ritz vectors
            collapsed = true;
            for (int r = 0; r < nroots; ++r)
                hipLaunchKernelGGL((k_scale_copy<double, T>), dim3(g), dim3(256), 0, d.s, X64 + int64_t(r) * N,
                                   B + int64_t(r) * N, 1.0, N);
            for (int r = 0; r < nroots; ++r)
                DV_TRY(hipMemcpyAsync(S + int64_t(r) * N, SX + int64_t(r) * N, N * es, hipMemcpyDeviceToDevice, d.s));
            for (int i = 0; i < max_space * max_space; ++i) G[i] = 0;
            for (int r = 0; r < nroots; ++r) G[size_t(r) * max_space + r] = theta[r];
            m = nroots;
        }
        // this iteration's Ritz vectors, for the next restart: after a collapse
        // onto them they are the first nroots basis vectors
        if (refined_now) {
            prev_ok = false;
        } else if (collapsed) {
            Yprev.assign(size_t(m) * nroots, 0.0);
            for (int r = 0; r < nroots; ++r) Yprev[size_t(r) * nroots + r] = 1.0;
            mprev = m;
            prev_ok = true;
        } else {
            Yprev.assign(size_t(m) * nroots, 0.0);
            for (int i = 0; i < m; ++i)
                for (int r = 0; r < nroots; ++r) Yprev[size_t(i) * nroots + r] = Y[size_t(i) * m + r];
            mprev = m;
            prev_ok = true;
        }
        DV_TRY(pspace_correct(theta));
        // (3) corrections, orthogonalised against the basis (classical Gram-Schmidt,
        // all corrections in one pass over the basis, repeated when cancellation asks
        // for it) and then against each other
        nnew = 0;
        bool any_open = false;
        for (int r = 0; r < nroots; ++r) any_open = any_open || refined_now || rnorm[r] > rtol;
        std::vector<int> cand;
        for (int r = 0; r < nroots && m + int(cand.size()) < max_space; ++r) {
            // roots whose residual already meets the threshold get no new direction
            if (any_open && !refined_now && rnorm[r] <= rtol) continue;
            cand.push_back(r);
        }
        const int nc = int(cand.size());
        if (nc > 0 && nc <= kMultiY) {
            // the corrections in TB slots 0..nc-1 (cand is increasing: cand[j] >= j)
            for (int j = 0; j < nc; ++j) {
                T *t = TB + int64_t(j) * N;
                if (cand[j] != j)
                    DV_TRY(hipMemcpyAsync(t, TB + int64_t(cand[j]) * N, N * es, hipMemcpyDeviceToDevice, d.s));
                if (par) DV_TRY(symmetrize(t));   // back onto the sector
            }
            // orthogonalised against the basis: one classical Gram-Schmidt pass, a
            // second one only when a correction lost more than half of its squared
            // norm to the first (the DGKS criterion); the same pass returns the Gram
            // matrix of the results
            std::vector<double> cc(size_t(std::max(m, 1)) * nc), pre(nc), pre2(nc), gram(size_t(nc) * nc);
            if (m > 0) DV_TRY(dots_multi(d, B, N, m, TB, N, nc, N, cc.data()));
            DV_TRY(subtract_gram(d, B, N, m, cc.data(), nc, TB, N, N, pre.data(), gram.data()));
            bool again = false;
            for (int j = 0; j < nc; ++j) again = again || gram[size_t(j) * nc + j] < 0.5 * pre[j];
            if (again && m > 0) {
                DV_TRY(dots_multi(d, B, N, m, TB, N, nc, N, cc.data()));
                DV_TRY(subtract_gram(d, B, N, m, cc.data(), nc, TB, N, N, pre2.data(), gram.data()));
            }
            // orthonormalised among themselves: Cholesky factor R of the Gram matrix
            // (G = R^T R), dropping a correction whose remaining norm is <= 1e-12;
            // the new basis vectors are T R^-1 over the kept ones, in one pass
            std::vector<double> R(size_t(nc) * nc, 0.0);
            std::vector<int> kept;
            for (int j = 0; j < nc; ++j) {
                for (size_t a = 0; a < kept.size(); ++a) {
                    const int k = kept[a];
                    double v = gram[size_t(k) * nc + j];
                    for (size_t b = 0; b < a; ++b) v -= R[size_t(kept[b]) * nc + k] * R[size_t(kept[b]) * nc + j];
                    R[size_t(k) * nc + j] = v / R[size_t(k) * nc + k];
                }
                double v = gram[size_t(j) * nc + j];
                for (int k : kept) v -= R[size_t(k) * nc + j] * R[size_t(k) * nc + j];
                if (!(v > 1e-24)) continue;
                R[size_t(j) * nc + j] = std::sqrt(v);
                kept.push_back(j);
            }
            const int nk = int(kept.size());
            std::vector<double> wts(size_t(std::max(nk, 1)) * nc, 0.0);   // new vector a = sum_k T_k wts[a][k]
            for (int a = 0; a < nk; ++a) {
                std::vector<double> x(nk, 0.0);
                for (int b = a; b >= 0; --b) {
                    double v = b == a ? 1.0 : 0.0;
                    for (int c2 = b + 1; c2 <= a; ++c2) v -= R[size_t(kept[b]) * nc + kept[c2]] * x[c2];
                    x[b] = v / R[size_t(kept[b]) * nc + kept[b]];
                }
                for (int b = 0; b <= a; ++b) wts[size_t(a) * nc + kept[b]] = x[b];
            }
            DV_TRY(combine_new(d, TB, N, nc, wts.data(), nk, B + int64_t(m) * N, N, N));
            nnew = nk;
        } else {
            for (int j = 0; j < nc; ++j) {
                T *t = B + int64_t(m + j) * N;
                DV_TRY(hipMemcpyAsync(t, TB + int64_t(cand[j]) * N, N * es, hipMemcpyDeviceToDevice, d.s));
                if (par) DV_TRY(symmetrize(t));   // back onto the sector
            }
            if (nc > 0 && m > 0) {
                std::vector<double> cc(size_t(m) * nc);
                for (int pass = 0; pass < 2; ++pass) {
                    DV_TRY(dots_multi(d, B, N, m, B + int64_t(m) * N, N, nc, N, cc.data()));
                    DV_TRY(subtract_multi(d, B, N, m, cc.data(), nc, B + int64_t(m) * N, N, N));
                }
            }
            for (int j = 0; j < nc; ++j) {
                T *t = B + int64_t(m + j) * N;
                for (int pass = 0; pass < 2 && nnew > 0; ++pass) {
                    DV_TRY(dots(d, B + int64_t(m) * N, N, nnew, t, N, col.data()));
                    DV_TRY(hipMemcpyAsync(d.dvec, col.data(), nnew * sizeof(double), hipMemcpyHostToDevice, d.s));
                    hipLaunchKernelGGL((k_subtract<T>), dim3(g), dim3(256), 0, d.s, B + int64_t(m) * N, N, nnew, d.dvec, t, N);
                }
                double tt;
                DV_TRY(dots(d, t, N, 1, t, N, &tt));
                const double nt = std::sqrt(tt);
                if (!(nt > 1e-12)) continue;
                T *dst = B + int64_t(m + nnew) * N;
                hipLaunchKernelGGL((k_scale_copy<T, T>), dim3(g), dim3(256), 0, d.s, t, dst, 1.0 / nt, N);
                ++nnew;
            }
        }
        if (nnew == 0) {
            // every correction vanished: the residuals lie in the basis (a basis
            // spanning the whole space or sector, or roots already at their
            // residual threshold); one more pass settles the convergence test
            bool small = true;
            for (int r = 0; r < nroots; ++r) small = small && rnorm[r] <= rtol;
            if (stalled || !(small || m >= dim)) break;
            stalled = true;
        } else {
            stalled = false;
        }
    }
    if (vecs && !x_fresh) DV_TRY(ritz_all(m, Y, false, true));   // no collapse since the last eigensolve
    DV_TRY(hipStreamSynchronize(d.s));
    for (int r = 0; r < nroots; ++r) energies[r] = (mixed && have_rq) ? erq[r] : theta[r];
    double rfinal = 0;
    for (int r = 0; r < nroots; ++r) rfinal = std::max(rfinal, (mixed && have_rq) ? r64[r] : rnorm[r]);
    if (vecs) {
        for (int r = 0; r < nroots; ++r) {
            T *dst = static_cast<T *>(vecs) + int64_t(r) * N;
            hipLaunchKernelGGL((k_scale_copy<double, T>), dim3(g), dim3(256), 0, d.s, X64 + int64_t(r) * N, dst, 1.0, N);
        }
        DV_TRY(hipStreamSynchronize(d.s));
    }
    if (stats) {
        stats->iterations = iter;
        stats->sigma_fp32 = nsig32;
        stats->sigma_fp64 = nsig64;
        stats->refinements = nref;
        stats->residual = rfinal;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!converged) return cis_set_error(ctx, CISIGMA_ENOCONV, "davidson: not converged within max_iter");
    return CISIGMA_OK;
}

}  // namespace

int davidson(cisigma_ctx *ctx, int nroots, double tol, double *energies, void *vecs, cisigma_stats *stats) {
    if (ctx->precision == CISIGMA_FP32) return run<float>(ctx, nroots, tol, energies, vecs, stats);
    return run<double>(ctx, nroots, tol, energies, vecs, stats);
}

}  // namespace cis
