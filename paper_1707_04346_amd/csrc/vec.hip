// vec.hip -- layout conversion, fill and diagonal kernels.
//
// The caller's CI vector holds blocks (alpha type, beta type) row-major
// [I_alpha][I_beta] (Sec. 3.1 TTSS blocks).  The sigma kernels work on two
// padded copies: alpha-major (rows = alpha strings, for sigma_2 and sigma_3)
// and beta-major (rows = beta strings, for sigma_1), so that every pass reads
// whole, aligned rows.  scatter_in makes both copies in one read of C (a
// 64x64 LDS-tiled transpose); gather_out forms
// sigma = alpha-major accumulator + (beta-major accumulator)^T.
#include "internal.h"

namespace cis {

namespace {

template <typename T>
__global__ void k_fill(T *x, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) x[i] = T(0);
}

// tiles: (block, r0, c0) with 64x64 extent; 256 threads
template <typename T>
__global__ __launch_bounds__(256) void k_scatter_in(const T *__restrict__ C, T *__restrict__ cp, T *__restrict__ ct,
                                                   const BlockDev *__restrict__ blk, const int *__restrict__ tb,
                                                   const int *__restrict__ tr, const int *__restrict__ tc) {
    __shared__ T tile[64][65];
    const int t = blockIdx.x;
    const BlockDev B = blk[tb[t]];
    const int r0 = tr[t], c0 = tc[t];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll 4
    for (int i = 0; i < 16; ++i) {
        int r = r0 + 4 * i + ty, c = c0 + tx;
        T v = 0;
        if (r < B.na && c < B.nb) {
            v = C[B.off + int64_t(r) * B.nb + c];
            cp[B.sega + int64_t(r) * B.lda + c] = v;
        }
        tile[4 * i + ty][tx] = v;
    }
    if (ct == nullptr) return;                 // the beta-major copy is not wanted (uniform)
    __syncthreads();
#pragma unroll 4
    for (int i = 0; i < 16; ++i) {
        int rb = c0 + 4 * i + ty, ca = r0 + tx;   // beta row, alpha column
        if (rb < B.nb && ca < B.na) ct[B.segb + int64_t(rb) * B.ldb + ca] = tile[tx][4 * i + ty];
    }
}

// M_S = 0 sector (one block, nalpha = nbeta, so both spins share the alpha
// layout): sigma = sp + st + p st^T, with st the alpha-alpha part and sp the
// alpha-beta part (Sec. 3.3: the beta-beta part of such a vector is the
// transposed alpha-alpha part).
template <typename T>
__global__ __launch_bounds__(256) void k_gather_parity(const T *__restrict__ sp, const T *__restrict__ st,
                                                      T *__restrict__ sig, const BlockDev *__restrict__ blk,
                                                      const int *__restrict__ tr, const int *__restrict__ tc,
                                                      T p) {
    __shared__ T tile[64][65];
    const int t = blockIdx.x;
    const BlockDev B = blk[0];
    const int r0 = tr[t], c0 = tc[t];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll 4
    for (int i = 0; i < 16; ++i) {
        int rr = c0 + 4 * i + ty, cc = r0 + tx;   // element (c, r) of the output tile
        T v = 0;
        if (rr < B.na && cc < B.nb) v = st[B.sega + int64_t(rr) * B.lda + cc];
        tile[tx][4 * i + ty] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int i = 0; i < 16; ++i) {
        int r = r0 + 4 * i + ty, c = c0 + tx;
        if (r < B.na && c < B.nb) {
            const int64_t a = B.sega + int64_t(r) * B.lda + c;
            sig[B.off + int64_t(r) * B.nb + c] = sp[a] + st[a] + p * tile[4 * i + ty][tx];
        }
    }
}

// The same for spaces with several blocks whose alpha and beta sides mirror each
// other: the transposed alpha-alpha part of block (ta, tb) is read from block
// (tb, ta) of st (both in the alpha-major layout).
template <typename T>
__global__ __launch_bounds__(256) void k_gather_parity_blocks(const T *__restrict__ sp, const T *__restrict__ st,
                                                             T *__restrict__ sig, const BlockDev *__restrict__ blk,
                                                             const int *__restrict__ tb, const int *__restrict__ tr,
                                                             const int *__restrict__ tc, const int *__restrict__ pblk,
                                                             T p) {
    __shared__ T tile[64][65];
    const int t = blockIdx.x;
    const BlockDev B = blk[tb[t]], Bp = blk[pblk[tb[t]]];
    const int r0 = tr[t], c0 = tc[t];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll 4
    for (int i = 0; i < 16; ++i) {
        int rr = c0 + 4 * i + ty, cc = r0 + tx;   // element (c, r) of the output tile, in the mirror block
        T v = 0;
        if (rr < Bp.na && cc < Bp.nb) v = st[Bp.sega + int64_t(rr) * Bp.lda + cc];
        tile[tx][4 * i + ty] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int i = 0; i < 16; ++i) {
        int r = r0 + 4 * i + ty, c = c0 + tx;
        if (r < B.na && c < B.nb) {
            const int64_t a = B.sega + int64_t(r) * B.lda + c;
            sig[B.off + int64_t(r) * B.nb + c] = sp[a] + st[a] + p * tile[4 * i + ty][tx];
        }
    }
}

// x <- (x + p x^T) / 2 in place on a caller-layout vector whose blocks mirror
// each other: element (r, c) of block b = (ta, tb) pairs with element (c, r) of
// block (tb, ta).  The 64x64 tile (b, r0, c0) is done together with its mirror by
// the tile with b < mirror, or on a diagonal block by the tile with r0 <= c0.
template <typename T>
__global__ __launch_bounds__(256) void k_symmetrize_blocks(T *x, const BlockDev *__restrict__ blk,
                                                          const int *__restrict__ tb, const int *__restrict__ tr,
                                                          const int *__restrict__ tc, const int *__restrict__ pblk,
                                                          T p) {
    __shared__ T a[64][65], bt[64][65];
    const int t = blockIdx.x, b = tb[t], b2 = pblk[b];
    const int r0 = tr[t], c0 = tc[t];
    if (b > b2 || (b == b2 && r0 > c0)) return;
    const BlockDev B = blk[b], M = blk[b2];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int r = r0 + i, c = c0 + tx;
        a[i][tx] = (r < B.na && c < B.nb) ? x[B.off + int64_t(r) * B.nb + c] : T(0);
        const int r2 = c0 + i, c2 = r0 + tx;          // mirror tile: rows c0.., columns r0..
        bt[i][tx] = (r2 < M.na && c2 < M.nb) ? x[M.off + int64_t(r2) * M.nb + c2] : T(0);
    }
    __syncthreads();
    // a[i][j] = x_b(r0 + i, c0 + j), bt[j][i] = x_b2(c0 + j, r0 + i)
    for (int i = ty; i < 64; i += 4) {
        const int r = r0 + i, c = c0 + tx;
        const T v = T(0.5) * (a[i][tx] + p * bt[tx][i]);
        if (r < B.na && c < B.nb) x[B.off + int64_t(r) * B.nb + c] = v;
        // mirror element x_b2(c0 + i, r0 + tx) = p * new x_b(r0 + tx, c0 + i)
        const int r2 = c0 + i, c2 = r0 + tx;
        const bool same = b == b2 && r0 == c0;         // a diagonal tile holds its own mirror
        if (!same && r2 < M.na && c2 < M.nb) x[M.off + int64_t(r2) * M.nb + c2] = p * T(0.5) * (a[tx][i] + p * bt[i][tx]);
    }
}

// x <- (x + p x^T) / 2 on x[n][n] row-major, in place: block (bi, bj) with
// bi <= bj owns the 32x32 tile pair (bi, bj) / (bj, bi); blocks below the
// diagonal return at once.
template <typename T>
__global__ __launch_bounds__(256) void k_symmetrize(T *x, int n, int nt, T p) {
    __shared__ T a[32][33], b[32][33];
    const int bi = blockIdx.x / nt, bj = blockIdx.x % nt;
    if (bi > bj) return;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 8 rows per pass
    const int r0 = bi * 32, c0 = bj * 32;
    for (int i = ty; i < 32; i += 8) {
        const int r = r0 + i, c = c0 + tx;
        a[i][tx] = (r < n && c < n) ? x[int64_t(r) * n + c] : T(0);
        const int r2 = c0 + i, c2 = r0 + tx;
        b[i][tx] = (r2 < n && c2 < n) ? x[int64_t(r2) * n + c2] : T(0);
    }
    __syncthreads();
    // a[i][j] = x(r0+i, c0+j), b[j][i] = x(c0+j, r0+i)
    for (int i = ty; i < 32; i += 8) {
        const int r = r0 + i, c = c0 + tx;
        const T v = T(0.5) * (a[i][tx] + p * b[tx][i]);
        if (r < n && c < n) x[int64_t(r) * n + c] = v;
        // the mirrored element x(c0+i, r0+tx) = p * new x(r0+tx, c0+i)
        const int r2 = c0 + i, c2 = r0 + tx;
        if (r2 < n && c2 < n && bi != bj) x[int64_t(r2) * n + c2] = p * T(0.5) * (a[tx][i] + p * b[i][tx]);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather_out(const T *__restrict__ sp, const T *__restrict__ st,
                                                   T *__restrict__ sig, const BlockDev *__restrict__ blk,
                                                   const int *__restrict__ tb, const int *__restrict__ tr,
                                                   const int *__restrict__ tc) {
    __shared__ T tile[64][65];
    const int t = blockIdx.x;
    const BlockDev B = blk[tb[t]];
    const int r0 = tr[t], c0 = tc[t];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll 4
    for (int i = 0; i < 16; ++i) {
        int rb = c0 + 4 * i + ty, ca = r0 + tx;
        T v = 0;
        if (rb < B.nb && ca < B.na) v = st[B.segb + int64_t(rb) * B.ldb + ca];
        tile[tx][4 * i + ty] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int i = 0; i < 16; ++i) {
        int r = r0 + 4 * i + ty, c = c0 + tx;
        if (r < B.na && c < B.nb)
            sig[B.off + int64_t(r) * B.nb + c] = sp[B.sega + int64_t(r) * B.lda + c] + tile[4 * i + ty][tx];
    }
}

// H_II = A_a(Ia) + A_b(Ib) + sum_{p in Ia, q in Ib} (pp|qq)
__global__ __launch_bounds__(256) void k_hdiag(double *out, const BlockDev *__restrict__ blk, const int *tb,
                                               const int *tr, const int *tc, const uint32_t *astr,
                                               const uint32_t *bstr, const int *astart, const int *bstart,
                                               const double *aa, const double *ab, const double *jpq, int n) {
    const int t = blockIdx.x;
    const BlockDev B = blk[tb[t]];
    const int r0 = tr[t], c0 = tc[t];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = 0; i < 16; ++i) {
        int r = r0 + 4 * i + ty, c = c0 + tx;
        if (r >= B.na || c >= B.nb) continue;
        int Ia = astart[B.ta] + r, Ib = bstart[B.tb] + c;
        uint32_t xa = astr[Ia], xb = bstr[Ib];
        double e = aa[Ia] + ab[Ib];
        for (uint32_t a = xa; a; a &= a - 1) {
            int pp = __ffs(a) - 1;
            for (uint32_t b = xb; b; b &= b - 1) e += jpq[pp * n + __ffs(b) - 1];
        }
        out[B.off + int64_t(r) * B.nb + c] = e;
    }
}

}  // namespace

hipError_t launch_fill(void *x, int64_t n, int dtype, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (dtype == CISIGMA_FP32)
        hipLaunchKernelGGL(k_fill<float>, dim3(unsigned(blocks)), dim3(256), 0, s, static_cast<float *>(x), n);
    else
        hipLaunchKernelGGL(k_fill<double>, dim3(unsigned(blocks)), dim3(256), 0, s, static_cast<double *>(x), n);
    return hipGetLastError();
}

hipError_t launch_scatter_in(const cisigma_ctx *ctx, const void *C, void *cp, void *ct, int dtype, hipStream_t s) {
    BlockTilesDev bt = block_tiles(ctx);
    if (bt.ntiles == 0) return hipSuccess;
    if (dtype == CISIGMA_FP32)
        hipLaunchKernelGGL(k_scatter_in<float>, dim3(bt.ntiles), dim3(256), 0, s, static_cast<const float *>(C),
                           static_cast<float *>(cp), static_cast<float *>(ct), bt.blk, bt.tb, bt.tr, bt.tc);
    else
        hipLaunchKernelGGL(k_scatter_in<double>, dim3(bt.ntiles), dim3(256), 0, s, static_cast<const double *>(C),
                           static_cast<double *>(cp), static_cast<double *>(ct), bt.blk, bt.tb, bt.tr, bt.tc);
    return hipGetLastError();
}

hipError_t launch_gather_out(const cisigma_ctx *ctx, const void *sp, const void *st, void *sigma, int dtype,
                             hipStream_t s) {
    BlockTilesDev bt = block_tiles(ctx);
    if (bt.ntiles == 0) return hipSuccess;
    if (dtype == CISIGMA_FP32)
        hipLaunchKernelGGL(k_gather_out<float>, dim3(bt.ntiles), dim3(256), 0, s, static_cast<const float *>(sp),
                           static_cast<const float *>(st), static_cast<float *>(sigma), bt.blk, bt.tb, bt.tr, bt.tc);
    else
        hipLaunchKernelGGL(k_gather_out<double>, dim3(bt.ntiles), dim3(256), 0, s, static_cast<const double *>(sp),
                           static_cast<const double *>(st), static_cast<double *>(sigma), bt.blk, bt.tb, bt.tr,
                           bt.tc);
    return hipGetLastError();
}

hipError_t launch_gather_parity(const cisigma_ctx *ctx, const void *sp, const void *st, void *sigma, int parity,
                                int dtype, hipStream_t s) {
    BlockTilesDev bt = block_tiles(ctx);
    if (bt.ntiles == 0) return hipSuccess;
    if (!ctx->cas) {
        if (!ctx->d_pblk) return hipErrorInvalidValue;
        if (dtype == CISIGMA_FP32)
            hipLaunchKernelGGL(k_gather_parity_blocks<float>, dim3(bt.ntiles), dim3(256), 0, s,
                               static_cast<const float *>(sp), static_cast<const float *>(st),
                               static_cast<float *>(sigma), bt.blk, bt.tb, bt.tr, bt.tc, ctx->d_pblk, float(parity));
        else
            hipLaunchKernelGGL(k_gather_parity_blocks<double>, dim3(bt.ntiles), dim3(256), 0, s,
                               static_cast<const double *>(sp), static_cast<const double *>(st),
                               static_cast<double *>(sigma), bt.blk, bt.tb, bt.tr, bt.tc, ctx->d_pblk,
                               double(parity));
        return hipGetLastError();
    }
    if (dtype == CISIGMA_FP32)
        hipLaunchKernelGGL(k_gather_parity<float>, dim3(bt.ntiles), dim3(256), 0, s, static_cast<const float *>(sp),
                           static_cast<const float *>(st), static_cast<float *>(sigma), bt.blk, bt.tr, bt.tc,
                           float(parity));
    else
        hipLaunchKernelGGL(k_gather_parity<double>, dim3(bt.ntiles), dim3(256), 0, s,
                           static_cast<const double *>(sp), static_cast<const double *>(st),
                           static_cast<double *>(sigma), bt.blk, bt.tr, bt.tc, double(parity));
    return hipGetLastError();
}

hipError_t launch_symmetrize(void *x, int n, int parity, int dtype, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int nt = (n + 31) / 32;
    const int64_t blocks = int64_t(nt) * nt;
    if (blocks > (int64_t(1) << 31) - 1) return hipErrorInvalidValue;
    if (dtype == CISIGMA_FP32)
        hipLaunchKernelGGL(k_symmetrize<float>, dim3(unsigned(blocks)), dim3(256), 0, s, static_cast<float *>(x), n, nt,
                           float(parity));
    else
        hipLaunchKernelGGL(k_symmetrize<double>, dim3(unsigned(blocks)), dim3(256), 0, s, static_cast<double *>(x), n,
                           nt, double(parity));
    return hipGetLastError();
}

hipError_t launch_symmetrize_blocks(const cisigma_ctx *ctx, void *x, int parity, int dtype, hipStream_t s) {
    BlockTilesDev bt = block_tiles(ctx);
    if (bt.ntiles == 0) return hipSuccess;
    if (!ctx->d_pblk) return hipErrorInvalidValue;
    if (dtype == CISIGMA_FP32)
        hipLaunchKernelGGL(k_symmetrize_blocks<float>, dim3(bt.ntiles), dim3(256), 0, s, static_cast<float *>(x), bt.blk,
                           bt.tb, bt.tr, bt.tc, ctx->d_pblk, float(parity));
    else
        hipLaunchKernelGGL(k_symmetrize_blocks<double>, dim3(bt.ntiles), dim3(256), 0, s, static_cast<double *>(x),
                           bt.blk, bt.tb, bt.tr, bt.tc, ctx->d_pblk, double(parity));
    return hipGetLastError();
}

hipError_t launch_hdiag(const cisigma_ctx *ctx, double *out, hipStream_t s) {
    BlockTilesDev bt = block_tiles(ctx);
    if (bt.ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hdiag, dim3(bt.ntiles), dim3(256), 0, s, out, bt.blk, bt.tb, bt.tr, bt.tc, ctx->sp[0].d_str,
                       ctx->sp[1].d_str, ctx->d_tstart[0], ctx->d_tstart[1], ctx->sp[0].d_adiag,
                       ctx->sp[1].d_adiag, ctx->d_jpq, ctx->n);
    return hipGetLastError();
}

}  // namespace cis
