// Learned Davidson preconditioner: a per-determinant MLP (8 -> 64 -> 64 -> 1,
// tanh, FP32) that predicts the component of the correction vector from
// features of the determinant and of the current Ritz pair. Feature
// definitions, target and parameter layout:
//   f0 = tanh((d - theta)/4)            f4 = alpha electrons outside the lowest
//   f1 = asinh(r_I sqrt(N)/|r|)              n_alpha orbitals / max(1, min(na, n-na))
//   f2 = asinh(x_I sqrt(N))             f5 = the same for beta
//   f3 = asinh(-r_I/(d-theta) sqrt(N)/|r|)   f6 = popcount(Ia ^ Ib) / n
//                                       f7 = tanh((d - d_min)/4)
// with d = H_II, r = sigma(x) - theta x, N = determinant count; target
// t_I = (x* - x)_I sqrt(N)/|x* - x| for the converged vector x* of the same
// root. Parameters: W1[8][64], b1[64], W2[64][64], b2[64], W3[64], b3.
#include "internal.h"

namespace casci {

constexpr int MD = MLP_IN, MH = MLP_HIDDEN;
constexpr int OW1 = 0, OB1 = OW1 + MD * MH, OW2 = OB1 + MH, OB2 = OW2 + MH * MH, OW3 = OB2 + MH,
              OB3 = OW3 + MH;
static_assert(OB3 + 1 == MLP_NPARAM, "parameter layout");

struct FeatIn {
    const double* diag;
    const double* x;
    const double* sx;
    double theta, rnorm, sqrtN, dmin;
    const uint64_t* astr;
    const uint64_t* bstr;
    int64_t Nb;
    int n, na, nb;
};

__device__ inline void mlp_features(const FeatIn& q, int64_t i, float f[MD], double* r_out, double* den_out)
{
    const double d = q.diag[i], xi = q.x[i];
    const double r = q.sx[i] - q.theta * xi;
    double den = d - q.theta;
    if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
    const double rs = q.rnorm > 0 ? q.sqrtN / q.rnorm : 0.0;
    const int64_t ia = i / q.Nb, ib = i - ia * q.Nb;
    const uint64_t a = q.astr[ia], b = q.bstr[ib];
    const uint64_t aufa = q.na >= 64 ? ~0ull : ((1ull << q.na) - 1);
    const uint64_t aufb = q.nb >= 64 ? ~0ull : ((1ull << q.nb) - 1);
    const int mina = q.na < q.n - q.na ? q.na : q.n - q.na;
    const int minb = q.nb < q.n - q.nb ? q.nb : q.n - q.nb;
    f[0] = (float)tanh((d - q.theta) / 4.0);
    f[1] = (float)asinh(r * rs);
    f[2] = (float)asinh(xi * q.sqrtN);
    f[3] = (float)asinh(-r / den * rs);
    f[4] = (float)__popcll(a & ~aufa) / (float)(mina > 1 ? mina : 1);
    f[5] = (float)__popcll(b & ~aufb) / (float)(minb > 1 ? minb : 1);
    f[6] = (float)__popcll(a ^ b) / (float)q.n;
    f[7] = (float)tanh((d - q.dmin) / 4.0);
    if (r_out) *r_out = r;
    if (den_out) *den_out = den;
}

// forward pass of one sample; weights are uniform across the wave (scalar loads)
__device__ inline float mlp_forward(const float* __restrict__ P, const float f[MD])
{
    float a1[MH];
#pragma unroll
    for (int j = 0; j < MH; ++j) {
        float z = P[OB1 + j];
#pragma unroll
        for (int k = 0; k < MD; ++k) z += f[k] * P[OW1 + k * MH + j];
        a1[j] = tanhf(z);
    }
    float y = P[OB3];
#pragma unroll 4
    for (int j = 0; j < MH; ++j) {
        float z = P[OB2 + j];
#pragma unroll
        for (int i = 0; i < MH; ++i) z += a1[i] * P[OW2 + i * MH + j];
        y += tanhf(z) * P[OW3 + j];
    }
    return y;
}

// learned correction for every determinant: t_I = network output
__global__ __launch_bounds__(256) void k_mlp_correction(FeatIn q, const float* __restrict__ P, int64_t N,
                                                       double* __restrict__ t)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        float f[MD];
        mlp_features(q, i, f, nullptr, nullptr);
        t[i] = (double)mlp_forward(P, f);
    }
}

// features (and targets when xstar != null) of the sampled determinants idx[0..m)
__global__ void k_mlp_collect(FeatIn q, const int64_t* __restrict__ idx, int m,
                              const double* __restrict__ xstar, double xsign, double dnorm_inv,
                              float* __restrict__ F, float* __restrict__ T)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= m) return;
    const int64_t i = idx[s];
    float f[MD];
    mlp_features(q, i, f, nullptr, nullptr);
#pragma unroll
    for (int k = 0; k < MD; ++k) F[(int64_t)s * MD + k] = f[k];
    if (T) T[s] = (float)((xsign * xstar[i] - q.x[i]) * q.sqrtN * dnorm_inv);
}

__global__ void k_mlp_forward_batch(const float* __restrict__ P, const float* __restrict__ X, int64_t N,
                                    float* __restrict__ Y)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < N; s += stride) {
        float f[MD];
#pragma unroll
        for (int k = 0; k < MD; ++k) f[k] = X[s * MD + k];
        Y[s] = mlp_forward(P, f);
    }
}

// ---------------------------------------------------------------------------
// training: per-block partial gradients of L = (1/Ntot) sum (y - t)^2 over the
// samples perm[begin + b*per .. ), 64 samples at a time, layer by layer in LDS.
// partial[b][0..NPARAM) = gradient, partial[b][NPARAM] = sum of squared errors.
// ---------------------------------------------------------------------------
constexpr int MB = 64;  // samples per block iteration

__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ P, const float* __restrict__ X,
                                                 const float* __restrict__ T, const int32_t* __restrict__ perm,
                                                 int64_t begin, int64_t count, int64_t per_block,
                                                 float inv_total, float* __restrict__ partial)
{
    __shared__ float sW[MLP_NPARAM];
    __shared__ float sX[MB][MD];
    __shared__ float A1[MB][MH + 1];
    __shared__ float A2[MB][MH + 1];
    __shared__ float D2[MB][MH + 1];
    __shared__ float D1[MB][MH + 1];
    __shared__ float sDy[MB];
    __shared__ float sE[MB];
    const int tid = threadIdx.x;
    for (int i = tid; i < MLP_NPARAM; i += 256) sW[i] = P[i];
    const int row = tid >> 2, cq = (tid & 3) * 16;   // 64 x 64 outputs: 16 per thread
    const int k1 = tid >> 5, j1 = (tid & 31) * 2;    // W1 gradient: 2 per thread
    float gW2[16], gW1[2] = {0.f, 0.f}, gv = 0.f, gb3 = 0.f, sse = 0.f;
    float gb1 = 0.f, gb2 = 0.f, gW3 = 0.f;
#pragma unroll
    for (int q = 0; q < 16; ++q) gW2[q] = 0.f;
    (void)gv;
    const int64_t b0 = begin + (int64_t)blockIdx.x * per_block;
    const int64_t b1end = min(b0 + per_block, begin + count);
    __syncthreads();
    for (int64_t c0 = b0; c0 < b1end; c0 += MB) {
        const int nvalid = (int)min((int64_t)MB, b1end - c0);
        for (int i = tid; i < MB * MD; i += 256) {
            const int s = i / MD, k = i - s * MD;
            sX[s][k] = s < nvalid ? X[(int64_t)perm[c0 + s] * MD + k] : 0.f;
        }
        __syncthreads();
        // layer 1
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int j = cq + q;
            float z = sW[OB1 + j];
#pragma unroll
            for (int k = 0; k < MD; ++k) z += sX[row][k] * sW[OW1 + k * MH + j];
            A1[row][j] = tanhf(z);
        }
        __syncthreads();
        // layer 2
#pragma unroll 4
        for (int q = 0; q < 16; ++q) {
            const int j = cq + q;
            float z = sW[OB2 + j];
            for (int i = 0; i < MH; ++i) z += A1[row][i] * sW[OW2 + i * MH + j];
            A2[row][j] = tanhf(z);
        }
        __syncthreads();
        // output and its loss gradient
        if (tid < MB) {
            float y = sW[OB3];
            for (int j = 0; j < MH; ++j) y += A2[tid][j] * sW[OW3 + j];
            const bool ok = tid < nvalid;
            const float e = ok ? y - T[perm[c0 + tid]] : 0.f;
            sDy[tid] = 2.f * e * inv_total;
            sE[tid] = e * e;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int j = cq + q;
            const float a = A2[row][j];
            D2[row][j] = sDy[row] * sW[OW3 + j] * (1.f - a * a);
        }
        __syncthreads();
#pragma unroll 4
        for (int q = 0; q < 16; ++q) {
            const int i = cq + q;
            float z = 0.f;
            for (int j = 0; j < MH; ++j) z += D2[row][j] * sW[OW2 + i * MH + j];
            const float a = A1[row][i];
            D1[row][i] = z * (1.f - a * a);
        }
        __syncthreads();
        // gradient accumulation (fixed order over the samples of the chunk)
        for (int s = 0; s < MB; ++s) {
            const float a1 = A1[s][row];
#pragma unroll
            for (int q = 0; q < 16; ++q) gW2[q] += a1 * D2[s][cq + q];
            gW1[0] += sX[s][k1] * D1[s][j1];
            gW1[1] += sX[s][k1] * D1[s][j1 + 1];
        }
        if (tid < MH) {
            float b1s = 0.f, b2s = 0.f, w3s = 0.f;
            for (int s = 0; s < MB; ++s) {
                b1s += D1[s][tid];
                b2s += D2[s][tid];
                w3s += A2[s][tid] * sDy[s];
            }
            gb1 += b1s;
            gb2 += b2s;
            gW3 += w3s;
        }
        if (tid == 0) {
            float b3s = 0.f, es = 0.f;
            for (int s = 0; s < MB; ++s) {
                b3s += sDy[s];
                es += sE[s];
            }
            gb3 += b3s;
            sse += es;
        }
        __syncthreads();
    }
    float* out = partial + (int64_t)blockIdx.x * (MLP_NPARAM + 1);
#pragma unroll
    for (int q = 0; q < 16; ++q) out[OW2 + row * MH + cq + q] = gW2[q];
    out[OW1 + k1 * MH + j1] = gW1[0];
    out[OW1 + k1 * MH + j1 + 1] = gW1[1];
    if (tid < MH) {
        out[OB1 + tid] = gb1;
        out[OB2 + tid] = gb2;
        out[OW3 + tid] = gW3;
    }
    if (tid == 0) {
        out[OB3] = gb3;
        out[MLP_NPARAM] = sse;
    }
}

// grad[p] = sum over blocks (fixed order, FP64 accumulation); slot NPARAM = sse
__global__ void k_mlp_reduce(const float* __restrict__ partial, int nblocks, float* __restrict__ grad,
                             double* __restrict__ sse)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > MLP_NPARAM) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial[(int64_t)b * (MLP_NPARAM + 1) + p];
    if (p < MLP_NPARAM) grad[p] = (float)s;
    else *sse = s;
}

__global__ void k_adam(float* __restrict__ P, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.f - b1) * gp;
    const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    P[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
static FeatIn feat_in(const MlpFeatArgs& a)
{
    FeatIn q;
    q.diag = a.diag;
    q.x = a.x;
    q.sx = a.sx;
    q.theta = a.theta;
    q.rnorm = a.rnorm;
    q.sqrtN = sqrt((double)a.N);
    q.dmin = a.dmin;
    q.astr = a.astr;
    q.bstr = a.bstr;
    q.Nb = a.Nb;
    q.n = a.n;
    q.na = a.na;
    q.nb = a.nb;
    return q;
}

hipError_t launch_mlp_correction(const MlpFeatArgs& a, const float* P, double* t, hipStream_t st)
{
    int64_t g = (a.N + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_mlp_correction, dim3((unsigned)g), dim3(256), 0, st, feat_in(a), P, a.N, t);
    return hipGetLastError();
}

hipError_t launch_mlp_collect(const MlpFeatArgs& a, const int64_t* idx, int m, const double* xstar,
                              double xsign, double dnorm_inv, float* F, float* T, hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_collect, dim3((m + 127) / 128), dim3(128), 0, st, feat_in(a), idx, m, xstar,
                       xsign, dnorm_inv, F, T);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* P, const float* X, int64_t N, float* Y, hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    int64_t g = (N + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_mlp_forward_batch, dim3((unsigned)g), dim3(256), 0, st, P, X, N, Y);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* P, const float* X, const float* T, const int32_t* perm,
                           int64_t begin, int64_t count, int64_t total, float* partial, int nblocks,
                           float* grad, double* sse, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    int64_t per = (count + nblocks - 1) / nblocks;
    per = (per + MB - 1) / MB * MB;
    const int used = (int)((count + per - 1) / per);
    hipLaunchKernelGGL(k_mlp_grad, dim3(used), dim3(256), 0, st, P, X, T, perm, begin, count, per,
                       1.0f / (float)total, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 1 + 255) / 256), dim3(256), 0, st, partial, used,
                       grad, sse);
    return hipGetLastError();
}

hipError_t launch_adam(float* P, const float* g, float* m, float* v, float lr, int step, hipStream_t st)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, P, g, m, v, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

}  // namespace casci
