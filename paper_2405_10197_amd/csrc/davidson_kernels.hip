// Davidson-Liu kernels (Sec. II.A.1 of the paper names the method; the
// paper gives no algorithmic detail). All reductions are two-stage with a
// fixed partition and a fixed summation order, so FP64 results are
// bitwise reproducible from run to run.
#include "internal.h"

namespace casci {

constexpr int RED_BLOCKS = 512;  // most stage-1 partials per output

// stage-1 blocks for vectors of length len: about 4096 elements per block
// (short vectors: launch-bound, fewer partials), at most RED_BLOCKS. The
// count depends on len only, so every sum is taken in the same order.
static int red_blocks(int64_t len)
{
    return (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(8, (len + 4095) / 4096));
}
constexpr int RED_THREADS = 256;

__device__ inline double block_sum(double v, double* sh)
{
    // fixed-order tree over RED_THREADS values
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// stage 1: partial[(i*nb + j) * nblk + xb] over a 4x4 group of (i, j), for
// x-block xb of nblk. The 1-D grid is laid out so that the workgroups of one
// x-block (all its (i, j) groups) run on the same XCD one after another: the
// vectors they share are then read from that XCD's L2 instead of from HBM
// once per group. Workgroup w runs on XCD w % 8.
__global__ __launch_bounds__(RED_THREADS) void k_block_dot(const double* __restrict__ A, int64_t lda,
                                                           int na, const double* __restrict__ B,
                                                           int64_t ldb, int nb, int64_t len, int nblk,
                                                           int gj, int ngrp, double* __restrict__ work)
{
    __shared__ double sh[RED_THREADS];
    const int w = blockIdx.x;
    const int loc = w / 8;
    const int xb = (loc / ngrp) * 8 + w % 8;
    if (xb >= nblk) return;
    const int g = loc % ngrp;
    const int i0 = (g / gj) * 4, j0 = (g % gj) * 4;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    const int64_t stride = (int64_t)nblk * blockDim.x;
    for (int64_t x = (int64_t)xb * blockDim.x + threadIdx.x; x < len; x += stride) {
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = (i0 + i < na) ? A[(int64_t)(i0 + i) * lda + x] : 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = (j0 + j < nb) ? B[(int64_t)(j0 + j) * ldb + x] : 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double s = block_sum(acc[i][j], sh);
            if (threadIdx.x == 0 && i0 + i < na && j0 + j < nb)
                work[((int64_t)(i0 + i) * nb + (j0 + j)) * nblk + xb] = s;
        }
}

// stage 1 for tall A (na >= 16, even length and strides): groups of 16 rows
// of A x 4 rows of B, two adjacent elements per lane (16-byte loads), so B is
// re-read a quarter as often; each wave sums a partial with a fixed xor tree,
// the four waves are added in a fixed order. Same grid layout and partials as
// k_block_dot. Measured at CAS(16,16) length, na = 48, nb = 4: 12.2 ms
// against 16.2 ms.
__global__ __launch_bounds__(RED_THREADS) void k_block_dot16(const double* __restrict__ A, int64_t lda, int na,
                                                             const double* __restrict__ B, int64_t ldb, int nb,
                                                             int64_t len, int nblk, int gj, int ngrp,
                                                             double* __restrict__ work)
{
    constexpr int GA = 16;
    __shared__ double sh[RED_THREADS / 64][GA * 4];
    const int w = blockIdx.x;
    const int loc = w / 8;
    const int xb = (loc / ngrp) * 8 + w % 8;
    if (xb >= nblk) return;
    const int g = loc % ngrp;
    const int i0 = (g / gj) * GA, j0 = (g % gj) * 4;
    double acc[GA][4];
#pragma unroll
    for (int i = 0; i < GA; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    const int64_t n2 = len / 2;
    const int64_t stride = (int64_t)nblk * blockDim.x;
    const double2 z = make_double2(0.0, 0.0);
    for (int64_t x = (int64_t)xb * blockDim.x + threadIdx.x; x < n2; x += stride) {
        double2 a[GA], b[4];
#pragma unroll
        for (int i = 0; i < GA; ++i)
            a[i] = (i0 + i < na) ? reinterpret_cast<const double2*>(A + (int64_t)(i0 + i) * lda)[x] : z;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            b[j] = (j0 + j < nb) ? reinterpret_cast<const double2*>(B + (int64_t)(j0 + j) * ldb)[x] : z;
#pragma unroll
        for (int i = 0; i < GA; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] += a[i].x * b[j].x + a[i].y * b[j].y;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < GA; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double s = acc[i][j];
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
            if (lane == 0) sh[wv][i * 4 + j] = s;
        }
    __syncthreads();
    if ((int)threadIdx.x < GA * 4) {
        const int i = threadIdx.x / 4, j = threadIdx.x % 4;
        const double s = (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
        if (i0 + i < na && j0 + j < nb) work[((int64_t)(i0 + i) * nb + (j0 + j)) * nblk + xb] = s;
    }
}

// stage 2: one wave per output (four per workgroup); lane l sums partials
// l, l + 64, ... in order, then a fixed xor tree over the lanes (the result
// does not depend on timing)
__global__ __launch_bounds__(256) void k_reduce_partials(const double* __restrict__ work, int nout, int nparts,
                                                         double* __restrict__ out)
{
    const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (o >= nout) return;  // uniform per wave
    double s = 0.0;
    for (int k = lane; k < nparts; k += 64) s += work[(int64_t)o * nparts + k];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) out[o] = s;
}

hipError_t launch_reduce_partials(const double* work, int nout, int nparts, double* out, hipStream_t st)
{
    if (nout <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_partials, dim3((nout + 3) / 4), dim3(256), 0, st, work, nout, nparts, out);
    return hipGetLastError();
}

hipError_t launch_block_dot(const double* A, int64_t lda, int na, const double* B, int64_t ldb,
                            int nb, int64_t len, double* work, double* out, hipStream_t st)
{
    if (na <= 0 || nb <= 0) return hipSuccess;
    const int nblk = red_blocks(len);
    const bool tall = na >= 16 && len % 2 == 0 && lda % 2 == 0 && ldb % 2 == 0 &&
                      ((uintptr_t)A | (uintptr_t)B) % 16 == 0;
    const int gj = (nb + 3) / 4, ngrp = ((na + (tall ? 15 : 3)) / (tall ? 16 : 4)) * gj;
    const int64_t nwg = (int64_t)((nblk + 7) / 8) * 8 * ngrp;
    if (tall)
        hipLaunchKernelGGL(k_block_dot16, dim3((unsigned)nwg), dim3(RED_THREADS), 0, st, A, lda, na, B, ldb, nb, len,
                           nblk, gj, ngrp, work);
    else
        hipLaunchKernelGGL(k_block_dot, dim3((unsigned)nwg), dim3(RED_THREADS), 0, st, A, lda, na, B, ldb, nb, len,
                           nblk, gj, ngrp, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int nout = na * nb;
    hipLaunchKernelGGL(k_reduce_partials, dim3((nout + 3) / 4), dim3(256), 0, st, work, nout, nblk, out);
    return hipGetLastError();
}

// Y_j = beta Y_j + sum_i A_i coef[i*ldc + j]
__global__ __launch_bounds__(256) void k_combine(const double* __restrict__ A, int64_t lda, int na,
                                                 const double* __restrict__ coef, int ldc, int nc,
                                                 double beta, double* __restrict__ Y, int64_t ldy,
                                                 int64_t len)
{
    __shared__ double sc[64 * 8];
    for (int t = threadIdx.x; t < na * nc; t += blockDim.x) {
        int i = t / nc, j = t - i * nc;
        sc[t] = coef[i * ldc + j];
    }
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < len; x += stride) {
        double acc[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = 0.0;
        for (int i = 0; i < na; ++i) {
            const double a = A[(int64_t)i * lda + x];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (j < nc) acc[j] += a * sc[i * nc + j];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (j < nc) {
                double* y = Y + (int64_t)j * ldy + x;
                *y = (beta == 0.0 ? 0.0 : beta * *y) + acc[j];
            }
    }
}

// the same with two adjacent elements per lane (16-byte loads and stores),
// for many rows of A with even length and strides: 13.3 ms against 14.5 ms at
// CAS(16,16) length, na = 44, nc = 4 (slower for a handful of rows)
template <int NC>
__global__ __launch_bounds__(256) void k_combine_pair(const double* __restrict__ A, int64_t lda, int na,
                                                      const double* __restrict__ coef, int ldc, double beta,
                                                      double* __restrict__ Y, int64_t ldy, int64_t len)
{
    __shared__ double sc[64 * NC];
    for (int t = threadIdx.x; t < na * NC; t += blockDim.x) {
        int i = t / NC, j = t - i * NC;
        sc[t] = coef[i * ldc + j];
    }
    __syncthreads();
    const int64_t n2 = len / 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n2; x += stride) {
        double2 acc[NC];
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[j] = make_double2(0.0, 0.0);
        for (int i = 0; i < na; ++i) {
            const double2 a = reinterpret_cast<const double2*>(A + (int64_t)i * lda)[x];
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const double c = sc[i * NC + j];
                acc[j].x += a.x * c;
                acc[j].y += a.y * c;
            }
        }
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            double2* y = reinterpret_cast<double2*>(Y + (int64_t)j * ldy) + x;
            double2 o = acc[j];
            if (beta != 0.0) {
                const double2 p = *y;
                o.x += beta * p.x;
                o.y += beta * p.y;
            }
            *y = o;
        }
    }
}

static unsigned ew_grid(int64_t n)
{
    int64_t g = (n + 255) / 256;
    return (unsigned)(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

hipError_t launch_combine(const double* A, int64_t lda, int na, const double* coef, int ldc, int nc,
                          double beta, double* Y, int64_t ldy, int64_t len, hipStream_t st)
{
    if (nc <= 0 || len <= 0) return hipSuccess;
    if (na > 64) return hipErrorInvalidValue;
    const bool pair = na >= 16 && len % 2 == 0 && lda % 2 == 0 && ldy % 2 == 0 &&
                      ((uintptr_t)A | (uintptr_t)Y) % 16 == 0;
    for (int j0 = 0; j0 < nc; j0 += 8) {
        int n8 = nc - j0 < 8 ? nc - j0 : 8;
        if (pair) {
            const dim3 g(ew_grid(len / 2)), b(256);
            const double* c = coef + j0;
            double* y = Y + (int64_t)j0 * ldy;
            switch (n8) {
            case 1: hipLaunchKernelGGL(k_combine_pair<1>, g, b, 0, st, A, lda, na, c, ldc, beta, y, ldy, len); break;
            case 2: hipLaunchKernelGGL(k_combine_pair<2>, g, b, 0, st, A, lda, na, c, ldc, beta, y, ldy, len); break;
            case 3: hipLaunchKernelGGL(k_combine_pair<3>, g, b, 0, st, A, lda, na, c, ldc, beta, y, ldy, len); break;
            case 4: hipLaunchKernelGGL(k_combine_pair<4>, g, b, 0, st, A, lda, na, c, ldc, beta, y, ldy, len); break;
            case 5: hipLaunchKernelGGL(k_combine_pair<5>, g, b, 0, st, A, lda, na, c, ldc, beta, y, ldy, len); break;
            case 6: hipLaunchKernelGGL(k_combine_pair<6>, g, b, 0, st, A, lda, na, c, ldc, beta, y, ldy, len); break;
            case 7: hipLaunchKernelGGL(k_combine_pair<7>, g, b, 0, st, A, lda, na, c, ldc, beta, y, ldy, len); break;
            default: hipLaunchKernelGGL(k_combine_pair<8>, g, b, 0, st, A, lda, na, c, ldc, beta, y, ldy, len); break;
            }
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            continue;
        }
        hipLaunchKernelGGL(k_combine, dim3(ew_grid(len)), dim3(256), 0, st, A, lda, na, coef + j0,
                           ldc, n8, beta, Y + (int64_t)j0 * ldy, ldy, len);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

__device__ inline double safe_denominator(double d)
{
    // |H_II - theta| clamped to >= 1e-8, sign kept
    if (fabs(d) < 1e-8) return d < 0 ? -1e-8 : 1e-8;
    return d;
}

// stage 1 of residual norms and Olsen dots, one blockIdx.y per root
__global__ __launch_bounds__(RED_THREADS) void k_residual(const double* __restrict__ X,
                                                          const double* __restrict__ SX, int64_t ld,
                                                          const double* __restrict__ theta,
                                                          const double* __restrict__ diag,
                                                          int64_t len, double* __restrict__ work)
{
    __shared__ double sh[RED_THREADS];
    const int k = blockIdx.y;
    const double th = theta[k];
    const double* x = X + (int64_t)k * ld;
    const double* sx = SX + (int64_t)k * ld;
    double rr = 0.0, xr = 0.0, xx = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) {
        const double xi = x[i];
        const double r = sx[i] - th * xi;
        const double inv = 1.0 / safe_denominator(diag[i] - th);
        rr += r * r;
        xr += xi * inv * r;
        xx += xi * inv * xi;
    }
    double s0 = block_sum(rr, sh), s1 = block_sum(xr, sh), s2 = block_sum(xx, sh);
    if (threadIdx.x == 0) {
        work[((int64_t)k * 4 + 0) * gridDim.x + blockIdx.x] = s0;
        work[((int64_t)k * 4 + 1) * gridDim.x + blockIdx.x] = s1;
        work[((int64_t)k * 4 + 2) * gridDim.x + blockIdx.x] = s2;
        work[((int64_t)k * 4 + 3) * gridDim.x + blockIdx.x] = 0.0;
    }
}

hipError_t launch_residual(const double* X, const double* SX, int64_t ld, int k, const double* theta,
                           const double* diag, int64_t len, double* work, double* out,
                           hipStream_t st)
{
    if (k <= 0) return hipSuccess;
    const int nblk = red_blocks(len);
    hipLaunchKernelGGL(k_residual, dim3(nblk, k), dim3(RED_THREADS), 0, st, X, SX, ld, theta, diag, len, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_partials, dim3((4 * k + 3) / 4), dim3(256), 0, st, work, 4 * k, nblk, out);
    return hipGetLastError();
}

__global__ void k_precondition(const double* __restrict__ X, const double* __restrict__ SX,
                               double theta, double eps, const double* __restrict__ diag,
                               int64_t len, double* __restrict__ T)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) {
        const double xi = X[i];
        const double r = SX[i] - theta * xi;
        T[i] = (-r + eps * xi) / safe_denominator(diag[i] - theta);
    }
}

hipError_t launch_precondition(const double* X, const double* SX, double theta, double eps,
                               const double* diag, int64_t len, double* T, hipStream_t st)
{
    hipLaunchKernelGGL(k_precondition, dim3(ew_grid(len)), dim3(256), 0, st, X, SX, theta, eps, diag,
                       len, T);
    return hipGetLastError();
}

__global__ void k_scale(double* x, double a, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] *= a;
}

hipError_t launch_scale(double* x, double a, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale, dim3(ew_grid(n)), dim3(256), 0, st, x, a, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// position of the largest |x_i| (ties: the lowest index), for the phase of a
// converged vector: stage 1 takes one contiguous range per block, stage 2 one
// wave over the partials (both orders fixed)
// ---------------------------------------------------------------------------
__device__ inline void absmax_pick(double& a, int64_t& i, double b, int64_t j)
{
    // larger |x| wins; an equal one with a lower index wins
    if (b > a || (b == a && j < i)) {
        a = b;
        i = j;
    }
}

__global__ __launch_bounds__(RED_THREADS) void k_absmax_partial(const double* __restrict__ x, int64_t n,
                                                                int nblk, double* __restrict__ pv,
                                                                int64_t* __restrict__ pi)
{
    __shared__ double sv[RED_THREADS];
    __shared__ int64_t si[RED_THREADS];
    const int64_t per = (n + nblk - 1) / nblk;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(n, lo + per);
    double a = -1.0;
    int64_t ai = INT64_MAX;
    for (int64_t k = lo + threadIdx.x; k < hi; k += RED_THREADS) absmax_pick(a, ai, fabs(x[k]), k);
    sv[threadIdx.x] = a;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int st = RED_THREADS / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            double b = sv[threadIdx.x];
            int64_t bi = si[threadIdx.x];
            absmax_pick(b, bi, sv[threadIdx.x + st], si[threadIdx.x + st]);
            sv[threadIdx.x] = b;
            si[threadIdx.x] = bi;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pv[blockIdx.x] = sv[0];
        pi[blockIdx.x] = si[0];
    }
}

// out[0] = x at the position, out[1] = the position (as a double: exact below 2^53)
__global__ __launch_bounds__(64) void k_absmax_final(const double* __restrict__ x, const double* __restrict__ pv,
                                                     const int64_t* __restrict__ pi, int nblk,
                                                     double* __restrict__ out)
{
    double a = -1.0;
    int64_t ai = INT64_MAX;
    for (int b = threadIdx.x; b < nblk; b += 64) absmax_pick(a, ai, pv[b], pi[b]);
    for (int off = 32; off > 0; off >>= 1) {
        const double b = __shfl_xor(a, off);
        const int64_t bi = __shfl_xor(ai, off);
        absmax_pick(a, ai, b, bi);
    }
    if (threadIdx.x == 0) {
        out[0] = ai == INT64_MAX ? 0.0 : x[ai];
        out[1] = ai == INT64_MAX ? -1.0 : (double)ai;
    }
}

hipError_t launch_absmax(const double* x, int64_t n, double* work, double* out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int nblk = red_blocks(n);
    double* pv = work;
    int64_t* pi = reinterpret_cast<int64_t*>(work + RED_BLOCKS);
    hipLaunchKernelGGL(k_absmax_partial, dim3(nblk), dim3(RED_THREADS), 0, st, x, n, nblk, pv, pi);
    hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(64), 0, st, x, pv, pi, nblk, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// lowest entries of the diagonal (start vectors): min/max, a histogram over
// [min, max], then the entries of the lowest bins, which the host sorts
// ---------------------------------------------------------------------------
// per-block minimum and maximum over a contiguous slice (fixed partition)
__global__ __launch_bounds__(RED_THREADS) void k_minmax_partial(const double* __restrict__ x, int64_t n, int nblk,
                                                                double* __restrict__ out)
{
    __shared__ double smin[RED_THREADS], smax[RED_THREADS];
    const int64_t per = (n + nblk - 1) / nblk;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(n, lo + per);
    double a = INFINITY, b = -INFINITY;
    for (int64_t k = lo + threadIdx.x; k < hi; k += RED_THREADS) {
        a = fmin(a, x[k]);
        b = fmax(b, x[k]);
    }
    smin[threadIdx.x] = a;
    smax[threadIdx.x] = b;
    __syncthreads();
    for (int st = RED_THREADS / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + st]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[blockIdx.x] = smin[0];
        out[nblk + blockIdx.x] = smax[0];
    }
}

// bin of a value: the same expression in the histogram and the collection
__device__ inline int value_bin(double v, double lo, double inv_w, int nbins)
{
    const double t = (v - lo) * inv_w;
    return t < (double)nbins ? (t > 0.0 ? (int)t : 0) : nbins - 1;
}

// one histogram per workgroup in LDS (the values crowd into few bins, so
// global atomics per element would serialise), added to the global one at
// the end; nbins <= VALUE_HIST_MAXBINS
constexpr int VALUE_HIST_MAXBINS = 4096;
__global__ __launch_bounds__(256) void k_value_hist(const double* __restrict__ x, int64_t n, double lo,
                                                    double inv_w, int nbins, unsigned* __restrict__ hist)
{
    __shared__ unsigned sh[VALUE_HIST_MAXBINS];
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) sh[b] = 0u;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
        atomicAdd(&sh[value_bin(x[k], lo, inv_w, nbins)], 1u);
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += blockDim.x)
        if (sh[b]) atomicAdd(&hist[b], sh[b]);
}

// entries in bins <= bmax, in any order (the caller sorts them); at most cap
__global__ __launch_bounds__(256) void k_value_collect(const double* __restrict__ x, int64_t n, double lo,
                                                       double inv_w, int nbins, int bmax,
                                                       unsigned long long* __restrict__ count,
                                                       int64_t* __restrict__ idx, double* __restrict__ val,
                                                       int64_t cap)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const double v = x[k];
        if (value_bin(v, lo, inv_w, nbins) <= bmax) {
            const unsigned long long s = atomicAdd(count, 1ull);
            if ((int64_t)s < cap) {
                idx[s] = k;
                val[s] = v;
            }
        }
    }
}

hipError_t launch_minmax(const double* x, int64_t n, double* out, int* nblk_out, hipStream_t st)
{
    const int nblk = red_blocks(n);
    *nblk_out = nblk;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_minmax_partial, dim3(nblk), dim3(RED_THREADS), 0, st, x, n, nblk, out);
    return hipGetLastError();
}

hipError_t launch_value_hist(const double* x, int64_t n, double lo, double inv_w, int nbins, unsigned* hist,
                             hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (nbins < 1 || nbins > VALUE_HIST_MAXBINS) return hipErrorInvalidValue;
    const int64_t g = std::min<int64_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(k_value_hist, dim3((unsigned)g), dim3(256), 0, st, x, n, lo, inv_w, nbins, hist);
    return hipGetLastError();
}

hipError_t launch_value_collect(const double* x, int64_t n, double lo, double inv_w, int nbins, int bmax,
                                unsigned long long* count, int64_t* idx, double* val, int64_t cap, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_value_collect, dim3(ew_grid(n)), dim3(256), 0, st, x, n, lo, inv_w, nbins, bmax, count,
                       idx, val, cap);
    return hipGetLastError();
}

}  // namespace casci
