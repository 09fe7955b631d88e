// sigma = H C kernels (the sigma build of Sec. II.A.1 of the paper).
//
// With E_pq = E^a_pq + E^b_pq and k_pq = h_pq - 1/2 sum_r (pr|rq), the
// Hamiltonian of eq. (hamiltonian) splits as
//   H = V + F_a + F_b + sum_{pq,rs} (pq|rs) E^a_pq E^b_rs,
// where F_s = sum k_pq E^s_pq + 1/2 sum (pq|rs) E^s_pq E^s_rs acts on the
// strings of one spin only (it is H of the one-spin system). On the CI
// matrix C[Ia][Ib]:
//   sigma_aa(Ia,:)  = sum_J F_a(Ia,J) C(J,:)           -- whole-row gathers
//   sigma_bb        = (F_b C^T)^T                       -- same kernel on C^T
//   sigma_ab(Ia,Ib) = sum_{e in L1(Ia)} s_e sum_rs (p_e q_e|rs)
//                       sum_Jb <Ib|E_rs|Jb> C(J_e, Jb)   -- MFMA contraction
// With alpha creators left of beta creators the alpha and beta substitution
// signs factorise, so no extra phase appears in sigma_ab.
#include "internal.h"

namespace casci {

// ---------------------------------------------------------------------------
// same-spin gather: Y(I,:) = [acc ? Y : 0] + sum_e val(I,e) X(col(I,e),:) + shift X(I,:)
// ---------------------------------------------------------------------------
// One wave computes one row I over a strip of LPE columns. The row's list
// (col, val) is read 64 entries at a time, one per lane (coalesced), and
// broadcast with readlane; G = 64/LPE entries are gathered per wave-wide
// load, one per lane group, and the group partials are combined with xor
// shuffles at the end. Workgroups are remapped so that each XCD sweeps a
// contiguous range of column strips: all rows of a strip then share that
// XCD's L2 copy of the strip of X.
__device__ inline int bcast_i32(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ inline double bcast_f64(double v, int lane)
{
    int2 u = *reinterpret_cast<int2*>(&v);
    u.x = __builtin_amdgcn_readlane(u.x, lane);
    u.y = __builtin_amdgcn_readlane(u.y, lane);
    return *reinterpret_cast<double*>(&u);
}

template <typename T, int LPE>
__global__ __launch_bounds__(256) void k_ss_gather(const int32_t* __restrict__ col,
                                                   const double* __restrict__ val, int r,
                                                   int64_t nrows, int64_t ncols,
                                                   const T* __restrict__ X, T* __restrict__ Y,
                                                   double shift, int acc, int64_t nrowblk,
                                                   int64_t nitems)
{
    constexpr int G = 64 / LPE;
    const int64_t per_xcd = gridDim.x / 8;
    const int64_t t = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (t >= nitems) return;
    const int64_t strip = t / nrowblk;
    const int64_t rb = t - strip * nrowblk;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t I = rb * 4 + wave;
    if (I >= nrows) return;
    const int g = lane / LPE, li = lane % LPE;
    const int64_t c = strip * LPE + li;
    const bool cok = c < ncols;
    const int32_t* colI = col + I * (int64_t)r;
    const double* valI = val + I * (int64_t)r;
    double a0 = 0.0, a1 = 0.0;
    for (int base = 0; base < r; base += 64) {
        const int e = base + lane;
        const int cj = e < r ? colI[e] : 0;
        const double vj = e < r ? valI[e] : 0.0;
#pragma unroll
        for (int j = 0; j < 64; j += 2 * G) {
            // two independent accumulators for memory-level parallelism; lane
            // group g takes entries j+g and j+G+g (all readlanes are uniform)
            int J0 = bcast_i32(cj, j), J1 = bcast_i32(cj, j + G);
            double v0 = bcast_f64(vj, j), v1 = bcast_f64(vj, j + G);
#pragma unroll
            for (int q = 1; q < G; ++q) {
                const int Jq0 = bcast_i32(cj, j + q), Jq1 = bcast_i32(cj, j + G + q);
                const double vq0 = bcast_f64(vj, j + q), vq1 = bcast_f64(vj, j + G + q);
                J0 = g == q ? Jq0 : J0;
                J1 = g == q ? Jq1 : J1;
                v0 = g == q ? vq0 : v0;
                v1 = g == q ? vq1 : v1;
            }
            // entries past r carry v = 0 and J = 0 (a valid row): no branch needed
            if (cok) {
                a0 += v0 * (double)X[(int64_t)J0 * ncols + c];
                a1 += v1 * (double)X[(int64_t)J1 * ncols + c];
            }
        }
    }
    double a = a0 + a1;
#pragma unroll
    for (int off = LPE; off < 64; off <<= 1) a += __shfl_xor(a, off);
    if (g == 0 && cok) {
        const int64_t o = I * ncols + c;
        double y = a + shift * (double)X[o];
        if (acc) y += (double)Y[o];
        Y[o] = (T)y;
    }
}

template <typename T, int LPE>
static hipError_t ss_gather(const int32_t* col, const double* val, int r, int64_t nrows,
                            int64_t ncols, const T* X, T* Y, double shift, int acc, hipStream_t st)
{
    if (nrows <= 0 || ncols <= 0) return hipSuccess;
    const int64_t nrowblk = (nrows + 3) / 4;
    const int64_t nstrip = (ncols + LPE - 1) / LPE;
    const int64_t nitems = nrowblk * nstrip;
    const int64_t grid = (nitems + 7) / 8 * 8;
    if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_ss_gather<T, LPE>), dim3((unsigned)grid), dim3(256), 0, st, col, val, r,
                       nrows, ncols, X, Y, shift, acc, nrowblk, nitems);
    return hipGetLastError();
}

hipError_t launch_ss_gather_f64(const int32_t* col, const double* val, int r, int64_t nrows,
                                int64_t ncols, const double* X, double* Y, double shift, int acc,
                                hipStream_t st)
{
    return ss_gather<double, 32>(col, val, r, nrows, ncols, X, Y, shift, acc, st);
}

hipError_t launch_ss_gather_f32(const int32_t* col, const double* val, int r, int64_t nrows,
                                int64_t ncols, const float* X, float* Y, double shift, int acc,
                                hipStream_t st)
{
    return ss_gather<float, 64>(col, val, r, nrows, ncols, X, Y, shift, acc, st);
}

// ---------------------------------------------------------------------------
// transpose through a padded LDS tile
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const T* __restrict__ in, T* __restrict__ out,
                                                   int64_t rows, int64_t cols, int acc, double scale)
{
    __shared__ T tile[64][65];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        int64_t r = r0 + i, c = c0 + tx;
        if (r < rows && c < cols) tile[i][tx] = in[r * cols + c];
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        int64_t orow = c0 + i, ocol = r0 + tx;  // out is cols x rows
        if (orow < cols && ocol < rows) {
            double v = scale * (double)tile[tx][i];
            if (acc) v += (double)out[orow * rows + ocol];
            out[orow * rows + ocol] = (T)v;
        }
    }
}

hipError_t launch_transpose_f64(const double* in, double* out, int64_t rows, int64_t cols, int acc,
                                double scale, hipStream_t st)
{
    if (rows <= 0 || cols <= 0) return hipSuccess;
    dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((rows + 63) / 64));
    hipLaunchKernelGGL(k_transpose<double>, grid, dim3(256), 0, st, in, out, rows, cols, acc, scale);
    return hipGetLastError();
}

hipError_t launch_transpose_f32(const float* in, float* out, int64_t rows, int64_t cols, int acc,
                                hipStream_t st)
{
    if (rows <= 0 || cols <= 0) return hipSuccess;
    dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((rows + 63) / 64));
    hipLaunchKernelGGL(k_transpose<float>, grid, dim3(256), 0, st, in, out, rows, cols, acc, 1.0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// alpha-beta contraction on MFMA
// ---------------------------------------------------------------------------
// One workgroup owns one alpha string Ia (and one chunk [lo, lo+chunk) of
// the sigma row, kept in LDS). For every tile of TN beta strings Jb:
//   D(e, Jb)  = C(J_e, Jb),  e in L1(Ia)           (row gathers -> LDS)
//   T(m, Jb)  = sum_e A(m, e) D(e, Jb),             A(m,e) = s_e (p_e q_e|r_m s_m)
//             (one 16-row M tile per wave, 16x16x4 FP64 MFMA)
//   sigma(Ia, Ib) += sign * T(m, Jb) for Ib = E_{r s} Jb, scattered from the
//             accumulator registers into the LDS row with atomic adds.
// Pair rows m: r <= s when the integrals are symmetric in rs (T(rs) = T(sr);
// the one of E_rs / E_sr that does not vanish on Jb is applied), or all
// ordered (r, s) when an S^2 penalty (not rs-symmetric) is folded in.
typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int AB_TN = 64;
constexpr int AB_LDD = AB_TN + 2;

__device__ inline int rank32(uint64_t mask, const int* __restrict__ b32, int ldb)
{
    int r = 0, k = 1;
    while (mask) {
        int p = __builtin_ctzll(mask);
        r += b32[p * ldb + k];
        ++k;
        mask &= mask - 1;
    }
    return r;
}

// scatter target of pair (r, s) acting on Jb; returns -1 if the operator vanishes
__device__ inline int ab_target(uint64_t jb, int r, int s, int full, const int* b32, int ldb,
                                int jb_index, int* sign)
{
    const int orr = (jb >> r) & 1, oss = (jb >> s) & 1;
    *sign = 1;
    if (r == s) return orr ? jb_index : -1;
    if (full) {
        if (!oss || orr) return -1;  // E_rs needs s occupied, r empty
    } else {
        if (orr == oss) return -1;   // exactly one of r, s occupied
    }
    if (__popcll(jb & between_mask(r, s)) & 1) *sign = -1;
    return rank32(jb ^ (1ull << r) ^ (1ull << s), b32, ldb);
}

template <int KBMAX, int MT>
__global__ __launch_bounds__(1024) void k_ab_f64(AbParams p, const double* __restrict__ Vt,
                                                 const double* __restrict__ C,
                                                 double* __restrict__ sigma, int kb_count,
                                                 int64_t chunk, int nchunks)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int Kp = kb_count * 4;
    const int ldb = p.nb + 2;
    double* sig = reinterpret_cast<double*>(smem);
    double* Dt = sig + chunk;
    int* sJ = reinterpret_cast<int*>(Dt + (int64_t)Kp * AB_LDD);
    int* b32 = sJ + Kp;

    // XCD-aware order: consecutive alpha strings share most of their L1 rows
    const int64_t per_xcd = gridDim.x / 8;
    const int64_t t = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int64_t nitems = p.Na * nchunks;
    if (t >= nitems) return;
    const int64_t ia = t / nchunks;
    const int64_t lo = (t - ia * nchunks) * chunk;
    const int64_t hi = min(lo + chunk, p.Nb);

    const int tid = threadIdx.x, nth = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int nwaves = nth >> 6;

    for (int64_t i = tid; i < hi - lo; i += nth) sig[i] = 0.0;
    for (int i = tid; i < Kp; i += nth) sJ[i] = i < p.sa ? l1_index(p.la_j[ia * p.sa + i]) : 0;
    for (int i = tid; i < p.n * ldb; i += nth) {
        int pp = i / ldb, kk = i - pp * ldb;
        b32[i] = kk <= p.nb ? (int)p.binom[pp * (p.n + 1) + kk] : 0;
    }

    // 16x16x4 FP64 MFMA operands: lane holds A(m0 + lane%16, 4*kb + lane/16) and
    // B(4*kb + lane/16, lane%16)
    double afr[MT][KBMAX];
    int pr_r[MT][4], pr_s[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int m0 = (wave + mt * nwaves) * 16;
        const int m = m0 + (lane & 15);
#pragma unroll
        for (int kb = 0; kb < KBMAX; ++kb) {
            double v = 0.0;
            const int e = kb * 4 + (lane >> 4);
            if (kb < kb_count && e < p.sa && m < p.M) {
                const int32_t enc = p.la_j[ia * p.sa + e];
                const int pq = p.la_pq[ia * p.sa + e];
                const int pqi = (pq & 0xff) * p.n + (pq >> 8);
                v = Vt[(int64_t)pqi * p.Mp + m] * l1_sign(enc);
            }
            afr[mt][kb] = v;
        }
        // accumulator element v of a lane holds row 4*v + lane/16, column lane%16
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int mm = m0 + 4 * v + (lane >> 4);
            const int code = mm < p.M ? p.pairs[mm] : 0xffff;
            pr_r[mt][v] = mm < p.M ? (code & 0xff) : -1;
            pr_s[mt][v] = code >> 8;
        }
    }
    __syncthreads();

    for (int64_t j0 = 0; j0 < p.Nb; j0 += AB_TN) {
        // gather D tile: rows J_e of C, columns [j0, j0+TN)
        for (int i = tid; i < Kp * AB_TN; i += nth) {
            const int k = i / AB_TN, cidx = i - k * AB_TN;
            const int64_t jb = j0 + cidx;
            double v = 0.0;
            if (k < p.sa && jb < p.Nb) v = C[(int64_t)sJ[k] * p.Nb + jb];
            Dt[k * AB_LDD + cidx] = v;
        }
        __syncthreads();
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int mtile = wave + mt * nwaves;
            if (mtile * 16 >= p.Mp) continue;
            for (int ns = 0; ns < AB_TN / 16; ++ns) {
                const int64_t jcol = j0 + ns * 16 + (lane & 15);
                if (j0 + ns * 16 >= p.Nb) break;
                d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kb = 0; kb < KBMAX; ++kb) {
                    if (kb < kb_count) {
                        const double b = Dt[(kb * 4 + (lane >> 4)) * AB_LDD + ns * 16 + (lane & 15)];
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(afr[mt][kb], b, acc, 0, 0, 0);
                    }
                }
                if (jcol < p.Nb) {
                    const uint64_t jb = p.bstr[jcol];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if (pr_r[mt][v] < 0) continue;
                        int sg;
                        const int tgt = ab_target(jb, pr_r[mt][v], pr_s[mt][v], p.full, b32, ldb,
                                                  (int)jcol, &sg);
                        if (tgt >= lo && tgt < hi) atomicAdd(&sig[tgt - lo], sg * acc[v]);
                    }
                }
            }
        }
        __syncthreads();
    }
    double* srow = sigma + ia * p.Nb;
    for (int64_t i = tid; i < hi - lo; i += nth) srow[lo + i] += sig[i];
}

static int64_t ab_lds_bytes(const AbParams& p, int kb_count, int64_t chunk, int elt)
{
    return chunk * elt + (int64_t)kb_count * 4 * AB_LDD * 8 + kb_count * 4 * 4 +
           (int64_t)p.n * (p.nb + 2) * 4 + 64;
}

hipError_t launch_ab_f64(const AbParams& p, const double* Vt, const double* C, double* sigma,
                         hipStream_t st)
{
    if (p.Na <= 0 || p.Nb <= 0 || p.sa <= 0 || p.M <= 0) return hipSuccess;
    const int kb_count = (p.sa + 3) / 4;
    const int mtiles = p.Mp / 16;
    const int MT = mtiles > 16 ? 2 : 1;
    const int nwaves = (mtiles + MT - 1) / MT;
    if (nwaves > 16) return hipErrorInvalidValue;
    const int64_t lds_cap = 160 * 1024 - 1024;
    int64_t fixed = ab_lds_bytes(p, kb_count, 0, 8);
    int64_t chunk = (lds_cap - fixed) / 8;
    if (chunk < 256) return hipErrorInvalidValue;
    int nchunks = (int)((p.Nb + chunk - 1) / chunk);
    chunk = (p.Nb + nchunks - 1) / nchunks;
    const size_t lds = (size_t)ab_lds_bytes(p, kb_count, chunk, 8);
    const int64_t items = p.Na * nchunks;
    const int64_t grid = (items + 7) / 8 * 8;
    dim3 blk(64 * nwaves);
#define AB_CASE(KB, MTV)                                                                         \
    if (kb_count <= KB && MT == MTV) {                                                           \
        hipFuncSetAttribute((const void*)k_ab_f64<KB, MTV>,                                      \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);               \
        hipLaunchKernelGGL((k_ab_f64<KB, MTV>), dim3((unsigned)grid), blk, lds, st, p, Vt, C,    \
                           sigma, kb_count, chunk, nchunks);                                     \
        return hipGetLastError();                                                                \
    }
    AB_CASE(4, 1)
    AB_CASE(8, 1)
    AB_CASE(12, 1)
    AB_CASE(16, 1)
    AB_CASE(24, 1)
    AB_CASE(32, 1)
    AB_CASE(8, 2)
    AB_CASE(16, 2)
    AB_CASE(24, 2)
    AB_CASE(32, 2)
#undef AB_CASE
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// small elementwise helpers
// ---------------------------------------------------------------------------
__global__ void k_f64_to_f32(const double* __restrict__ in, float* __restrict__ out, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}
__global__ void k_f32_to_f64(const float* __restrict__ in, double* __restrict__ out, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (double)in[i];
}
__global__ void k_axpby(double a, const double* __restrict__ x, double b, double* __restrict__ y,
                        int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i] + b * y[i];
}

static unsigned ew_grid(int64_t n)
{
    int64_t g = (n + 255) / 256;
    return (unsigned)(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

hipError_t launch_convert_f64_to_f32(const double* in, float* out, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_f64_to_f32, dim3(ew_grid(n)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}
hipError_t launch_convert_f32_to_f64(const float* in, double* out, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_f32_to_f64, dim3(ew_grid(n)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}
hipError_t launch_axpby_f64(double a, const double* x, double b, double* y, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpby, dim3(ew_grid(n)), dim3(256), 0, st, a, x, b, y, n);
    return hipGetLastError();
}

hipError_t launch_ab_lowp(const AbParams&, int, const void*, const double*, double*, hipStream_t)
{
    return hipErrorNotSupported;
}

}  // namespace casci
