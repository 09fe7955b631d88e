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

#include <climits>

namespace casci {

static thread_local const char* g_launch_reason = "";
const char* launch_reason() { return g_launch_reason; }
void set_launch_reason(const char* why) { g_launch_reason = why; }

static hipError_t invalid(const char* why)
{
    g_launch_reason = why;
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// same-spin gather: Y(I,:) = [acc ? Y : 0] + sum_e val(I,e) X(col(I,e),:) + shift X(I,:)
// ---------------------------------------------------------------------------
// One wave computes one row I over a strip of LPE x VW columns (VW adjacent
// columns per lane, loaded as one vector). The row's list
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

template <typename T, int VW>
struct Vec;
template <typename T>
struct Vec<T, 1> {
    using type = T;
};
template <>
struct Vec<float, 2> {
    using type = float2;
};
template <>
struct Vec<double, 2> {
    using type = double2;
};

__device__ inline float bcast_val(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ inline double bcast_val(double v, int lane) { return bcast_f64(v, lane); }

template <typename TX, typename TY, int LPE, int VW, typename TC, typename TV>
__global__ __launch_bounds__(256) void k_ss_gather(const TC* __restrict__ col,
                                                   const TV* __restrict__ val, int r,
                                                   int64_t nrows, int64_t ncols,
                                                   const TX* __restrict__ X, int64_t ldx,
                                                   TY* __restrict__ Y, double shift, int acc,
                                                   int64_t nrowblk, int64_t nitems, int64_t ipw)
{
    constexpr int G = 64 / LPE;
    using VX = typename Vec<TX, VW>::type;
    const int64_t per_xcd = gridDim.x / 8;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane / LPE, li = lane % LPE;
    // The grid is capped (the launch size in work-items is a 32-bit quantity);
    // workgroup w takes the ipw consecutive items [w*ipw, (w+1)*ipw), w in XCD
    // order, so the workgroups running on one XCD still cover one stretch of
    // consecutive row blocks of the same strip.
    const int64_t w = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int64_t t_end = min(nitems, (w + 1) * ipw);
    for (int64_t t = w * ipw; t < t_end; ++t) {
        const int64_t strip = t / nrowblk;
        const int64_t rb = t - strip * nrowblk;
        const int64_t I = rb * 4 + wave;
        if (I >= nrows) continue;
        // this lane's VW consecutive columns (VW = 2 needs an even ldx: aligned pairs)
        const int64_t c = (strip * LPE + li) * VW;
        const bool full = c + VW <= ncols;
        const bool cok = c < ncols;
        const TC* colI = col + I * (int64_t)r;
        const TV* valI = val + I * (int64_t)r;
        auto load = [&](int J, double* out) {
            const TX* src = X + (int64_t)J * ldx + c;
            if constexpr (VW == 1) {
                out[0] = (double)*src;
            } else {
                if (full) {
                    const VX v = *reinterpret_cast<const VX*>(src);
                    out[0] = (double)v.x;
                    out[1] = (double)v.y;
                } else {
                    out[0] = (double)src[0];
                    out[1] = 0.0;
                }
            }
        };
        constexpr int NACC = 4;  // independent accumulators: loads in flight per wave
        double acc_[NACC][VW] = {};
        for (int base = 0; base < r; base += 64) {
            const int e = base + lane;
            const int cj = e < r ? (int)colI[e] : 0;
            const TV vj = e < r ? valI[e] : (TV)0;
#pragma unroll
            for (int j = 0; j < 64; j += NACC * G) {
                // lane group g takes entries j + h*G + g, h < NACC (readlanes are uniform)
                int J[NACC];
                double v[NACC];
#pragma unroll
                for (int h = 0; h < NACC; ++h) {
                    J[h] = bcast_i32(cj, j + h * G);
                    v[h] = (double)bcast_val(vj, j + h * G);
#pragma unroll
                    for (int q = 1; q < G; ++q) {
                        const int Jq = bcast_i32(cj, j + h * G + q);
                        const double vq = (double)bcast_val(vj, j + h * G + q);
                        J[h] = g == q ? Jq : J[h];
                        v[h] = g == q ? vq : v[h];
                    }
                }
                // entries past r carry v = 0 and J = 0 (a valid row): no branch needed
                if (cok) {
                    double x[NACC][VW];
#pragma unroll
                    for (int h = 0; h < NACC; ++h) load(J[h], x[h]);
#pragma unroll
                    for (int h = 0; h < NACC; ++h)
#pragma unroll
                        for (int u = 0; u < VW; ++u) acc_[h][u] += v[h] * x[h][u];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < VW; ++u) {
            double a = (acc_[0][u] + acc_[1][u]) + (acc_[2][u] + acc_[3][u]);
#pragma unroll
            for (int off = LPE; off < 64; off <<= 1) a += __shfl_xor(a, off);
            if (g == 0 && c + u < ncols) {
                const int64_t o = I * ncols + c + u;
                double y = a + shift * (double)X[I * ldx + c + u];
                if (acc) y += (double)Y[o];
                Y[o] = (TY)y;
            }
        }
    }
}

template <typename TX, typename TY, int LPE, int VW, typename TC, typename TV>
static hipError_t ss_gather(const TC* col, const TV* val, int r, int64_t nrows,
                            int64_t ncols, const TX* X, int64_t ldx, TY* Y, double shift, int acc,
                            hipStream_t st)
{
    if (nrows <= 0 || ncols <= 0) return hipSuccess;
    if (VW > 1 && ldx % VW != 0) return invalid("same-spin gather: paired columns need an even row stride");
    const int64_t nrowblk = (nrows + 3) / 4;
    const int64_t nstrip = (ncols + LPE * VW - 1) / (LPE * VW);
    const int64_t nitems = nrowblk * nstrip;
    // at most 2^22 workgroups of 256 (each takes ipw consecutive items)
    const int64_t cap = (int64_t)1 << 22;
    const int64_t ipw = (nitems + cap - 1) / cap;
    const int64_t nwg = (nitems + ipw - 1) / ipw;
    const int64_t grid = (nwg + 7) / 8 * 8;
    hipLaunchKernelGGL((k_ss_gather<TX, TY, LPE, VW, TC, TV>), dim3((unsigned)grid), dim3(256), 0, st, col, val, r,
                       nrows, ncols, X, ldx, Y, shift, acc, nrowblk, nitems, ipw);
    return hipGetLastError();
}

// strip width code: 16 / 32 / 64 lanes per entry with one column each, or 128
// = 64 lanes with two adjacent columns each (needs an even row stride; an odd
// one falls back to 64)
template <typename TX, typename TY, typename TC, typename TV>
static hipError_t ss_gather_w(const TC* col, const TV* val, int r, int64_t nrows, int64_t ncols,
                              const TX* X, int64_t ldx, TY* Y, double shift, int acc, hipStream_t st, int lpe)
{
    switch (lpe) {
    case 16: return ss_gather<TX, TY, 16, 1>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
    case 32: return ss_gather<TX, TY, 32, 1>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
    case 0:
    case 64: return ss_gather<TX, TY, 64, 1>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
    case 128:
        if (ldx % 2 != 0) return ss_gather<TX, TY, 64, 1>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
        return ss_gather<TX, TY, 64, 2>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
    default: return invalid("same-spin gather: strip width code must be 16, 32, 64 or 128");
    }
}

hipError_t launch_ss_gather_f64(const SsOp& op, int64_t nrows, int64_t ncols, const double* X, double* Y,
                                double shift, int acc, hipStream_t st, int lpe)
{
    if (op.col16)
        return ss_gather_w<double, double>(op.col16, op.val, op.r, nrows, ncols, X, ncols, Y, shift, acc, st, lpe);
    return ss_gather_w<double, double>(op.col, op.val, op.r, nrows, ncols, X, ncols, Y, shift, acc, st, lpe);
}

hipError_t launch_ss_gather_f32in(const SsOp& op, int64_t nrows, int64_t ncols, const float* X, int64_t ldx,
                                  double* Y, double shift, int acc, hipStream_t st, int lpe)
{
    if (op.col16 && op.val32)
        return ss_gather_w<float, double>(op.col16, op.val32, op.r, nrows, ncols, X, ldx, Y, shift, acc, st, lpe);
    return ss_gather_w<float, double>(op.col, op.val, op.r, nrows, ncols, X, ldx, Y, shift, acc, st, lpe);
}

hipError_t launch_ss_gather_f32(const SsOp& op, int64_t nrows, int64_t ncols, const float* X, float* Y,
                                double shift, int acc, hipStream_t st, int lpe)
{
    if (op.col16 && op.val32)
        return ss_gather_w<float, float>(op.col16, op.val32, op.r, nrows, ncols, X, ncols, Y, shift, acc, st, lpe);
    return ss_gather_w<float, float>(op.col, op.val, op.r, nrows, ncols, X, ncols, Y, shift, acc, st, lpe);
}

// compact copies of an operator: 16-bit columns (N < 65536) and FP32 values
__global__ void k_compact_op(const int32_t* __restrict__ col, const double* __restrict__ val, int64_t n,
                             uint16_t* __restrict__ col16, float* __restrict__ val32)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        col16[i] = (uint16_t)col[i];
        val32[i] = (float)val[i];
    }
}

hipError_t launch_compact_op(const int32_t* col, const double* val, int64_t n, uint16_t* col16, float* val32,
                             hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t g = std::min<int64_t>((n + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(k_compact_op, dim3((unsigned)g), dim3(256), 0, st, col, val, n, col16, val32);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// S <- scale * (S + p S^T) in place for a square matrix (p = +-1): the tile
// pair (bi, bj) / (bj, bi) is read into LDS by one block before either is
// written, so every output uses the original values.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sym_add(double* __restrict__ S, int64_t n, double p,
                                                 double scale, int64_t nb, const double* __restrict__ T)
{
    __shared__ double A[32][33];
    __shared__ double B[32][33];
    // blockIdx.x enumerates pairs bi <= bj row by row; row bi starts at
    // s(bi) = bi nb - bi (bi - 1) / 2: invert the quadratic, then settle the
    // rounding with integer checks
    const int64_t k = blockIdx.x;
    auto rs = [nb](int64_t b) { return b * nb - b * (b - 1) / 2; };
    const double q = (double)(2 * nb + 1);
    int64_t bi = (int64_t)((q - sqrt(q * q - 8.0 * (double)k)) * 0.5);
    bi = bi < 0 ? 0 : (bi > nb - 1 ? nb - 1 : bi);
    while (bi > 0 && rs(bi) > k) --bi;
    while (bi + 1 < nb && rs(bi + 1) <= k) ++bi;
    const int64_t bj = bi + (k - rs(bi));
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t r0 = bi * 32, c0 = bj * 32;
    for (int i = ty; i < 32; i += 8) {
        const int64_t ra = r0 + i, ca = c0 + tx;
        A[i][tx] = (ra < n && ca < n) ? S[ra * n + ca] : 0.0;
        const int64_t rb = c0 + i, cb = r0 + tx;
        B[i][tx] = (rb < n && cb < n) ? S[rb * n + cb] : 0.0;
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        const int64_t ra = r0 + i, ca = c0 + tx;
        if (ra < n && ca < n)
            S[ra * n + ca] = scale * (A[i][tx] + p * B[tx][i]) + (T ? T[ra * n + ca] : 0.0);
        if (bi != bj) {
            const int64_t rb = c0 + i, cb = r0 + tx;
            if (rb < n && cb < n)
                S[rb * n + cb] = scale * (B[i][tx] + p * A[tx][i]) + (T ? T[rb * n + cb] : 0.0);
        }
    }
}

hipError_t launch_sym_add(double* S, int64_t n, int p, double scale, hipStream_t st, const double* T)
{
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 31) / 32;
    const int64_t pairs = nb * (nb + 1) / 2;
    if (pairs > 0x7fffffffLL) return invalid("sym_add: matrix too large");
    hipLaunchKernelGGL(k_sym_add, dim3((unsigned)pairs), dim3(256), 0, st, S, n, (double)p, scale, nb, T);
    return hipGetLastError();
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
// FP64 kernel (k_ab; the FP32/BF16 kernel below shares the contraction and
// replaces the atomic scatter). One workgroup owns one alpha string Ia (and
// one chunk [lo, lo+chunk) of the sigma row, accumulated in LDS). For every
// tile of TN beta strings Jb:
//   D(e, Jb)  = C(J_e, Jb),  e in L1(Ia)           (row gathers -> LDS)
//   T(m, Jb)  = sum_e A(m, e) D(e, Jb),             A(m,e) = s_e (p_e q_e|r_m s_m)
//             (one 16-row M tile per wave, 16x16xK MFMA, four N sub-tiles
//              as independent accumulator chains)
//   sigma(Ia, Ib) += sign * T(m, Jb) for Ib = E_{r s} Jb, scattered from the
//             accumulator registers into the LDS row with atomic adds.
// Pair rows m: r <= s when the integrals are symmetric in rs (T(rs) = T(sr);
// the one of E_rs / E_sr that does not vanish on Jb is applied), or all
// ordered (r, s) when an S^2 penalty (not rs-symmetric) is folded in.
// The scatter target of (m, Jb) does not depend on Ia, so it is tabulated once
// per string set: tg[Jb][m] = Ib with the sign folded in as in the lists
// (Ib or ~Ib), AB_NONE where E_rs Jb vanishes. Each lane reads the entries of
// exactly the accumulator elements it owns: the A rows are ordered so that a
// lane's four accumulator elements are four consecutive pair rows, i.e. one
// 16-byte load per 16-column sub-tile.
// The next tile of C and its targets are loaded into registers while the
// current one is multiplied, so the gather latency hides behind the MFMA work.
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef int i4 __attribute__((ext_vector_type(4)));

constexpr int32_t AB_NONE = INT32_MIN;  // tabulated target of a vanishing E_rs Jb

constexpr int AB_TN = 64;

struct MfmaF64 {
    using elem = double;   // element stored in the D tile
    using frag = double;   // MFMA operand of one lane
    using acc = d4;
    using lacc = double;   // LDS accumulator
    static constexpr int K = 4;
    static constexpr bool kmajor_tile = false;
    __device__ static acc mma(frag a, frag b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // accumulator element v of a lane holds row 4*v + lane/16, column lane%16;
    // A row r carries pair row 4*(r%4) + r/4 so that element v of a lane holds
    // pair row 4*(lane/16) + v
    __device__ static int arow(int r) { return 4 * (r & 3) + (r >> 2); }
    __device__ static elem cvt(double x) { return x; }
};

struct MfmaF32 {
    using elem = float;
    using frag = float;
    using acc = f4;
    using lacc = float;
    static constexpr int K = 4;
    static constexpr bool kmajor_tile = false;
    __device__ static acc mma(frag a, frag b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // accumulator element v of a lane holds row 4*(lane/16) + v
    __device__ static int arow(int r) { return r; }
    __device__ static elem cvt(double x) { return (float)x; }
};

struct MfmaBF16 {
    using elem = __bf16;
    using frag = bf8;
    using acc = f4;
    using lacc = float;
    static constexpr int K = 32;
    static constexpr bool kmajor_tile = true;  // tile stored [column][k]: 8 k per lane in one read
    __device__ static acc mma(frag a, frag b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static int arow(int r) { return r; }
    __device__ static elem cvt(double x) { return (__bf16)(float)x; }
};

template <typename MF>
struct TileLayout {
    // D tile of Kp rows (k) x TN columns. The [column][k] form shifts each
    // group of 8 columns by another 16 bytes: a wave's commit writes 8 columns
    // of 8 rows, and with the plain row stride (a multiple of 16 bytes) every
    // column group would land in the same LDS banks.
    __host__ __device__ static int size(int Kp) { return MF::kmajor_tile ? AB_TN * (Kp + 9) : Kp * (AB_TN + 2); }
    __device__ static int at(int k, int c, int Kp)
    {
        return MF::kmajor_tile ? c * (Kp + 8) + 8 * (c >> 3) + k : k * (AB_TN + 2) + c;
    }
};

// target and sign of the pair (r, s) acting on the beta string jb (column jcol)
__device__ inline int ab_lookup(uint64_t jb, int r, int s, int full, int n, int nb_el, int sb,
                                const int32_t* __restrict__ lb_j, int64_t jcol, int* sign)
{
    *sign = 1;
    const int orr = (jb >> r) & 1, oss = (jb >> s) & 1;
    if (r == s) return orr ? (int)jcol : -1;
    int a, b;
    if (full) {
        if (!oss || orr) return -1;  // E_rs needs s occupied, r empty
        a = s;
        b = r;
    } else {
        if (orr == oss) return -1;   // exactly one of r, s occupied
        a = oss ? s : r;
        b = oss ? r : s;
    }
    const uint64_t nmask = (n >= 64) ? ~0ull : ((1ull << n) - 1);
    const int pos = __popcll(jb & ((1ull << a) - 1)) * (n - nb_el + 1) +
                    __popcll(~jb & nmask & ((1ull << b) - 1)) + (a < b ? 1 : 0);
    const int32_t enc = lb_j[jcol * sb + pos];
    *sign = l1_sign(enc);
    return l1_index(enc);
}

// tg[j * Mp + m] for every beta string j and pair row m < Mp
__global__ __launch_bounds__(256) void k_ab_targets(AbParams p, int32_t* __restrict__ tg)
{
    const int64_t total = p.Nb * p.Mp;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = i / p.Mp;
        const int m = (int)(i - j * p.Mp);
        int32_t out = AB_NONE;
        if (m < p.M) {
            const int code = p.pairs[m];
            int sg;
            const int t = ab_lookup(p.bstr[j], code & 0xff, code >> 8, p.full, p.n, p.nb, p.sb, p.lb_j, j, &sg);
            if (t >= 0) out = l1_encode(t, sg);
        }
        tg[i] = out;
    }
}

hipError_t launch_ab_targets(const AbParams& p, int32_t* tg, hipStream_t st)
{
    if (p.Nb <= 0 || p.Mp <= 0) return hipSuccess;
    if (p.Mp % 16 != 0) return invalid("alpha-beta targets: pair rows not padded to 16");
    int64_t g = (p.Nb * p.Mp + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_ab_targets, dim3((unsigned)g), dim3(256), 0, st, p, tg);
    return hipGetLastError();
}

// targets of the accumulator elements a lane owns in one 64-column tile
template <int MT>
__device__ inline void ab_load_targets(const AbParams& p, int64_t j0, int wave, int nwaves, int lane,
                                       i4 (&dst)[MT][4])
{
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int m0 = (wave + mt * nwaves) * 16;
#pragma unroll
        for (int ns = 0; ns < 4; ++ns) {
            const int64_t jc = j0 + ns * 16 + (lane & 15);
            i4 v = {AB_NONE, AB_NONE, AB_NONE, AB_NONE};
            if (m0 < p.Mp && jc < p.Nb) v = *reinterpret_cast<const i4*>(p.tg + jc * p.Mp + m0 + 4 * (lane >> 4));
            dst[mt][ns] = v;
        }
    }
}

// scatter-add of one 16x64 accumulator block into the LDS row chunk [lo, hi)
template <typename LACC, typename ACC>
__device__ inline void ab_scatter(LACC* sig, const ACC (&acc)[4], const i4 (&tgt)[4], int64_t lo, int64_t hi)
{
#pragma unroll
    for (int ns = 0; ns < 4; ++ns) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int32_t e = tgt[ns][v];
            if (e != AB_NONE) {
                const int64_t tgi = l1_index(e);
                if (tgi >= lo && tgi < hi) {
                    const LACC x = (LACC)acc[ns][v];
                    atomicAdd(&sig[tgi - lo], e >= 0 ? x : -x);
                }
            }
        }
    }
}

constexpr int AB_MAX_WAVES = 12;

template <typename MF, int KBMAX, int MT, int PF>
__global__ __launch_bounds__(64 * AB_MAX_WAVES) void k_ab(AbParams p, const typename MF::elem* __restrict__ Vt,
                                             const double* __restrict__ C, double* __restrict__ sigma,
                                             int kb_count, int64_t chunk, int nchunks)
{
    using elem = typename MF::elem;
    using lacc = typename MF::lacc;
    using acc_t = typename MF::acc;
    extern __shared__ __align__(16) unsigned char smem[];
    const int Kp = kb_count * MF::K;
    lacc* sig = reinterpret_cast<lacc*>(smem);
    elem* Dt = reinterpret_cast<elem*>(smem + ((chunk * sizeof(lacc) + 15) / 16) * 16);
    int* sJ = reinterpret_cast<int*>(Dt + ((TileLayout<MF>::size(Kp) * (int)sizeof(elem) + 15) / 16) * 16 / sizeof(elem));

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

    for (int64_t i = tid; i < hi - lo; i += nth) sig[i] = (lacc)0;
    for (int i = tid; i < Kp; i += nth) sJ[i] = i < p.sa ? l1_index(p.la_j[ia * p.sa + i]) : 0;

    // A fragments (row lane%16 of each M tile carries pair row arow(lane%16))
    typename MF::frag afr[MT][KBMAX];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int m0 = (wave + mt * nwaves) * 16;
        const int m = m0 + MF::arow(lane & 15);
#pragma unroll
        for (int kb = 0; kb < KBMAX; ++kb) {
            typename MF::frag f;
            constexpr int PER = MF::K / 4;  // operand elements per lane
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int e = kb * MF::K + (lane >> 4) * PER + q;
                elem v = MF::cvt(0.0);
                if (kb < kb_count && e < p.sa && m < p.M) {
                    const int32_t enc = p.la_j[ia * p.sa + e];
                    const int pq = p.la_pq[ia * p.sa + e];
                    const int pqi = (pq & 0xff) * p.n + (pq >> 8);
                    v = Vt[(int64_t)pqi * p.Mp + m];
                    if (l1_sign(enc) < 0) v = -v;
                }
                if constexpr (PER == 1) f = v; else f[q] = v;
            }
            afr[mt][kb] = f;
        }
    }
    __syncthreads();

    const int tile_elems = Kp * AB_TN;
    double pf[PF];
    auto load_tile = [&](int64_t j0) {
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int idx = tid + i * nth;
            const int k = idx / AB_TN, c = idx - k * AB_TN;
            double v = 0.0;
            if (idx < tile_elems && k < p.sa && j0 + c < p.Nb) v = C[(int64_t)sJ[k] * p.Nb + j0 + c];
            pf[i] = v;
        }
    };
    auto store_tile = [&]() {
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int idx = tid + i * nth;
            if (idx < tile_elems) {
                const int k = idx / AB_TN, c = idx - k * AB_TN;
                Dt[TileLayout<MF>::at(k, c, Kp)] = MF::cvt(pf[i]);
            }
        }
    };
    load_tile(0);
    store_tile();
    __syncthreads();

    for (int64_t j0 = 0; j0 < p.Nb; j0 += AB_TN) {
        const bool more = j0 + AB_TN < p.Nb;
        // this tile's targets: their latency hides behind the FP64 MFMA chain
        i4 tgc[MT][4];
        ab_load_targets<MT>(p, j0, wave, nwaves, lane, tgc);
        if (more) load_tile(j0 + AB_TN);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int mtile = wave + mt * nwaves;
            if (mtile * 16 >= p.Mp) continue;
            acc_t acc[4];
#pragma unroll
            for (int ns = 0; ns < 4; ++ns)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[ns][v] = 0;
#pragma unroll
            for (int kb = 0; kb < KBMAX; ++kb) {
                if (kb < kb_count) {
#pragma unroll
                    for (int ns = 0; ns < 4; ++ns) {
                        typename MF::frag b;
                        const int c = ns * 16 + (lane & 15);
                        if constexpr (MF::kmajor_tile) {
                            b = *reinterpret_cast<const typename MF::frag*>(
                                &Dt[TileLayout<MF>::at(kb * MF::K + (lane >> 4) * (MF::K / 4), c, Kp)]);
                        } else {
                            b = Dt[TileLayout<MF>::at(kb * MF::K + (lane >> 4), c, Kp)];
                        }
                        acc[ns] = MF::mma(afr[mt][kb], b, acc[ns]);
                    }
                }
            }
            ab_scatter<lacc, acc_t>(sig, acc, tgc[mt], lo, hi);
        }
        __syncthreads();
        if (more) store_tile();
        __syncthreads();
    }
    double* srow = sigma + ia * p.Nb;
    if (p.overwrite)
        for (int64_t i = tid; i < hi - lo; i += nth) srow[lo + i] = (double)sig[i];
    else
        for (int64_t i = tid; i < hi - lo; i += nth) srow[lo + i] += (double)sig[i];
}

// ---------------------------------------------------------------------------
// low-precision alpha-beta contraction (FP32 or BF16 MFMA, FP32 accumulate)
// ---------------------------------------------------------------------------
// Same contraction as k_ab, with the scatter done without atomics. C is first
// converted once per sigma to the MFMA input type with its rows padded to a
// multiple of 16 bytes, so D tiles are gathered with 16-byte loads (a BF16
// tile row of 64 columns is one 128-byte line). Per 64-column tile:
//   1. MFMA: T(m, Jb) for all pair rows, written to an LDS tile Ts[Jb][m];
//   2. reduce: each lane owns one target Ib of the tile (from the grouped
//      table, see AbReduce) and adds the signed T entries of its group into
//      the FP32 sigma row in LDS with a plain read-add-write. A target occurs
//      once per tile, so no two lanes touch the same word, and every sum is
//      taken in a fixed order (the result is bitwise reproducible).
// The next tile's C segments and table block are loaded into registers while
// the current tile is multiplied and reduced.
constexpr int ABL_MAX_WAVES = 12;

template <typename MF, int KBMAX, int MT, int SPT, typename TO, int NS>
__global__ __launch_bounds__(64 * ABL_MAX_WAVES) void k_ab_lp(
    AbParams p, AbReduce r, const typename MF::elem* __restrict__ Vt,
    const typename MF::elem* __restrict__ Cs, int64_t ldc, TO* __restrict__ sigma, int kb_count,
    int64_t chunk, int nchunks)
{
    using elem = typename MF::elem;
    using acc_t = typename MF::acc;
    using vec_t = uint4;  // 16 bytes
    constexpr int VEC = 16 / sizeof(elem);
    constexpr int SEGS = AB_TN / VEC;  // 16-byte segments per tile row
    extern __shared__ __align__(16) unsigned char smem[];
    const int Kp = kb_count * MF::K;
    const int tsz = ((TileLayout<MF>::size(Kp) * (int)sizeof(elem) + 15) / 16) * 16;
    const int ldT = r.ldT;
    const int zslot = AB_TN * ldT;
    float* sig = reinterpret_cast<float*>(smem);
    unsigned char* base = smem + ((chunk * 4 + 15) / 16) * 16;
    elem* Dt = reinterpret_cast<elem*>(base);
    float* Ts = reinterpret_cast<float*>(base + tsz);
    unsigned char* Tab = base + tsz + (((int64_t)zslot + 4) * 4 + 15) / 16 * 16;
    int* sJ = reinterpret_cast<int*>(Tab + (int64_t)r.max_nseg * 16);

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

    for (int64_t i = tid; i < hi - lo; i += nth) sig[i] = 0.f;
    for (int i = tid; i < Kp; i += nth) sJ[i] = i < p.sa ? l1_index(p.la_j[ia * p.sa + i]) : -1;
    if (tid == 0) Ts[zslot] = 0.f;

    // Waves form 4/NS column groups (NS 16-column sub-tiles of the 64-column
    // tile each) x nwaves*NS/4 pair-row groups (MT consecutive 16-row M tiles
    // each): a wave reads only its columns of the D tile from LDS.
    constexpr int NG = 4 / NS;
    const int ngrp = wave % NG, mgrp = wave / NG;
    typename MF::frag afr[MT][KBMAX];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int m0 = (mgrp * MT + mt) * 16;
        const int m = m0 + MF::arow(lane & 15);
#pragma unroll
        for (int kb = 0; kb < KBMAX; ++kb) {
            typename MF::frag f;
            constexpr int PER = MF::K / 4;
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int e = kb * MF::K + (lane >> 4) * PER + q;
                elem v = MF::cvt(0.0);
                if (kb < kb_count && e < p.sa && m < p.M) {
                    const int32_t enc = p.la_j[ia * p.sa + e];
                    const int pq = p.la_pq[ia * p.sa + e];
                    v = Vt[(int64_t)((pq & 0xff) * p.n + (pq >> 8)) * p.Mp + m];
                    if (l1_sign(enc) < 0) v = -v;
                }
                if constexpr (PER == 1) f = v; else f[q] = v;
            }
            afr[mt][kb] = f;
        }
    }
    __syncthreads();

    // Segments of one tile: nseg of C (Kp rows x SEGS), then the tile's table
    // block. issue() starts the global loads into a register set; commit_d()
    // and commit_t() store a set to LDS once the current tile no longer needs
    // the buffer. Two register sets keep the loads of the next two tiles in
    // flight while the current one is multiplied and reduced.
    const int nseg = Kp * SEGS;
    const int64_t ntiles = (p.Nb + AB_TN - 1) / AB_TN;
    auto issue = [&](vec_t (&pf)[SPT], int64_t tile) {
        const int2 ti = r.tinfo[tile];
        const int64_t j0 = tile * AB_TN;
        const int tseg0 = ti.x, tnseg = ti.y & 0xfffff;
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int sidx = tid + q * nth;
            vec_t v = {0u, 0u, 0u, 0u};
            if (sidx < nseg) {
                const int k = sidx / SEGS, sg = sidx - k * SEGS;
                const int64_t col = j0 + sg * VEC;
                const int J = sJ[k];
                if (J >= 0 && col < ldc) v = *reinterpret_cast<const vec_t*>(Cs + J * ldc + col);
            } else if (sidx - nseg < tnseg) {
                v = r.tab[tseg0 + (sidx - nseg)];
            }
            pf[q] = v;
        }
    };
    auto commit_d = [&](const vec_t (&pf)[SPT]) {
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int sidx = tid + q * nth;
            if (sidx < nseg) {
                const int k = sidx / SEGS, sg = sidx - k * SEGS;
                const elem* ve = reinterpret_cast<const elem*>(&pf[q]);
#pragma unroll
                for (int e = 0; e < VEC; ++e) Dt[TileLayout<MF>::at(k, sg * VEC + e, Kp)] = ve[e];
            }
        }
    };
    auto commit_t = [&](const vec_t (&pf)[SPT], int tnseg) {
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int sidx = tid + q * nth;
            if (sidx >= nseg && sidx - nseg < tnseg)
                reinterpret_cast<vec_t*>(Tab)[sidx - nseg] = pf[q];
        }
    };
    // multiply and reduce the tile held in LDS; then commit the next one (in pfn)
    auto step = [&](int64_t tile, int nch, const vec_t (&pfn)[SPT], bool has_next, int nseg_next) {
        {
            acc_t acc[MT][NS];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int ns = 0; ns < NS; ++ns)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[mt][ns][v] = 0.f;
#pragma unroll
            for (int kb = 0; kb < KBMAX; ++kb) {
                if (kb < kb_count) {
#pragma unroll
                    for (int ns = 0; ns < NS; ++ns) {
                        const int c = (ngrp * NS + ns) * 16 + (lane & 15);
                        typename MF::frag b;
                        if constexpr (MF::kmajor_tile) {
                            b = *reinterpret_cast<const typename MF::frag*>(
                                &Dt[TileLayout<MF>::at(kb * MF::K + (lane >> 4) * (MF::K / 4), c, Kp)]);
                        } else {
                            b = Dt[TileLayout<MF>::at(kb * MF::K + (lane >> 4), c, Kp)];
                        }
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt)
                            if ((mgrp * MT + mt) * 16 < p.Mp) acc[mt][ns] = MF::mma(afr[mt][kb], b, acc[mt][ns]);
                    }
                }
            }
            // element v of this lane: pair row mtile*16 + 4*(lane/16) + v, column c
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int mtile = mgrp * MT + mt;
                if (mtile * 16 < p.Mp)
#pragma unroll
                    for (int ns = 0; ns < NS; ++ns) {
                        const int c = (ngrp * NS + ns) * 16 + (lane & 15);
                        *reinterpret_cast<f4*>(&Ts[c * ldT + mtile * 16 + 4 * (lane >> 4)]) = acc[mt][ns];
                    }
            }
        }
        __syncthreads();
        if (has_next) commit_d(pfn);
        {
            const uint16_t* wb = reinterpret_cast<const uint16_t*>(Tab);
            const int hsegs = (nwaves + 1 + 7) >> 3;
            const int dsegs = (nch + 3) >> 2;
            const uint32_t* dsc = reinterpret_cast<const uint32_t*>(Tab + hsegs * 16);
            const uint16_t* tgt = reinterpret_cast<const uint16_t*>(Tab + (hsegs + dsegs) * 16);
            const uint2* off = reinterpret_cast<const uint2*>(Tab + (hsegs + dsegs + nch * 8) * 16);
            const int qe = wb[wave + 1];
            for (int q = wb[wave]; q < qe; ++q) {
                const uint32_t d = dsc[q];
                const int cb = (int)(d & 0xfffff), nbk = (int)(d >> 20);
                const int tg = tgt[q * 64 + lane];
                float s = 0.f;
                for (int b = 0; b < nbk; ++b) {
                    const uint2 w = off[(cb + b) * 64 + lane];
                    const uint32_t o[4] = {w.x & 0xffffu, w.x >> 16, w.y & 0xffffu, w.y >> 16};
                    float v[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) v[u] = Ts[o[u] & 0x7fff];
#pragma unroll
                    for (int u = 0; u < 4; ++u) s += (o[u] & 0x8000) ? -v[u] : v[u];
                }
                if (tg != 0xffff && tg >= lo && tg < hi) sig[tg - lo] += s;
            }
        }
        __syncthreads();
        if (has_next) commit_t(pfn, nseg_next);
        (void)tile;
    };

    vec_t pfa[SPT], pfb[SPT];
    int2 ti0 = r.tinfo[0];
    int2 ti1 = {0, 0};
    issue(pfa, 0);
    if (ntiles > 1) {
        ti1 = r.tinfo[1];
        issue(pfb, 1);
    }
    commit_d(pfa);
    commit_t(pfa, ti0.y & 0xfffff);
    __syncthreads();
    int nch = ti0.y >> 20;
    // invariant at the top: tile t in LDS, tile t+1 in pfb (described by ti1)
    for (int64_t t = 0; t < ntiles; t += 2) {
        int2 ti2 = {0, 0};
        if (t + 2 < ntiles) {
            ti2 = r.tinfo[t + 2];
            issue(pfa, t + 2);
        }
        step(t, nch, pfb, t + 1 < ntiles, ti1.y & 0xfffff);
        if (t + 1 >= ntiles) break;
        nch = ti1.y >> 20;
        int2 ti3 = {0, 0};
        if (t + 3 < ntiles) {
            ti3 = r.tinfo[t + 3];
            issue(pfb, t + 3);
        }
        step(t + 1, nch, pfa, t + 2 < ntiles, ti2.y & 0xfffff);
        nch = ti2.y >> 20;
        ti1 = ti3;
    }
    __syncthreads();
    TO* srow = sigma + ia * p.Nb;
    if (p.overwrite)
        for (int64_t i = tid; i < hi - lo; i += nth) srow[lo + i] = (TO)sig[i];
    else
        for (int64_t i = tid; i < hi - lo; i += nth) srow[lo + i] = (TO)((double)srow[lo + i] + (double)sig[i]);
}

int abl_waves(int Mp)
{
    (void)Mp;
    return ABL_MAX_WAVES;  // 4 column groups x 3 pair-row groups
}

// layout of the low-precision kernel's waves: NS 16-column sub-tiles per wave
// (1: 4 column groups x 3 row groups; 4: one column group x 12 row groups)
// and MT 16-row M tiles per wave
// afr_regs: registers of one M tile's A fragments (kb_count operands). The
// column-group layout gives a wave up to four M tiles; when their fragments
// would take more than 64 registers (FP32 at n = 18: 4 x 23) the kernel
// spills, and the one-tile-per-wave layout is used instead.
static void abl_layout(int Mp, int afr_regs, int& NS, int& MT)
{
    const int mtiles = Mp / 16;
    const int mt3 = (mtiles + ABL_MAX_WAVES / 4 - 1) / (ABL_MAX_WAVES / 4);
    if (mtiles <= 4 * (ABL_MAX_WAVES / 4) && mt3 * afr_regs <= 64) {
        NS = 1;
        MT = (mtiles + ABL_MAX_WAVES / 4 - 1) / (ABL_MAX_WAVES / 4);
    } else {
        NS = 4;
        MT = (mtiles + ABL_MAX_WAVES - 1) / ABL_MAX_WAVES;
    }
}

template <typename MF>
static int64_t abl_lds_bytes(int kb_count, int ldT, int max_nseg, int64_t chunk)
{
    const int Kp = kb_count * MF::K;
    int64_t b = (chunk * 4 + 15) / 16 * 16;
    b += ((int64_t)TileLayout<MF>::size(Kp) * sizeof(typename MF::elem) + 15) / 16 * 16;
    b += (((int64_t)AB_TN * ldT + 4) * 4 + 15) / 16 * 16;
    b += (int64_t)max_nseg * 16;
    b += (int64_t)Kp * 4 + 64;
    return b;
}

template <typename MF, typename TO>
static hipError_t abl_launch(const AbParams& p, const AbReduce& r, const void* Vt, const void* Cs, int64_t ldc,
                             TO* sigma, hipStream_t st)
{
    if (p.Na <= 0 || p.Nb <= 0 || p.sa <= 0 || p.M <= 0) return hipSuccess;
    if (r.ldT < p.Mp + 4 || (int64_t)AB_TN * r.ldT + 1 > 0x7fff || r.ldT % 4 != 0)
        return invalid("alpha-beta: T tile stride does not fit the table's 15-bit offsets");
    if (p.Nb >= 0xffff) return invalid("alpha-beta: more than 65534 beta strings for the low-precision table");
    const int kb_count = (p.sa + MF::K - 1) / MF::K;
    const int nwaves = abl_waves(p.Mp);
    int NS = 1, MT = 1;
    abl_layout(p.Mp, kb_count * (int)(sizeof(typename MF::frag) / 4), NS, MT);
    if (NS == 4 && MT > 2) return invalid("alpha-beta: too many pair rows (norb too large)");
    const int64_t fixed = abl_lds_bytes<MF>(kb_count, r.ldT, r.max_nseg, 0);
    const int64_t cap = 160 * 1024 - 512;
    int64_t chunk = (cap - fixed) / 4;
    if (chunk < 256) return invalid("alpha-beta: LDS too small for the sigma row chunk");
    int nchunks = (int)((p.Nb + chunk - 1) / chunk);
    chunk = (p.Nb + nchunks - 1) / nchunks;
    const size_t lds = (size_t)abl_lds_bytes<MF>(kb_count, r.ldT, r.max_nseg, chunk);
    const int nseg = kb_count * MF::K * (AB_TN * (int)sizeof(typename MF::elem) / 16) + r.max_nseg;
    const int spt = (nseg + 64 * nwaves - 1) / (64 * nwaves);
    if (spt > 8) return invalid("alpha-beta: tile larger than the prefetch registers");
    const int64_t items = p.Na * nchunks;
    const int64_t grid = (items + 7) / 8 * 8;
    dim3 blk(64 * nwaves);
#define ABL_GO(KBV, MTV, SPTV, NSV)                                                                 \
    {                                                                                               \
        auto kern = k_ab_lp<MF, KBV, MTV, SPTV, TO, NSV>;                                           \
        hipError_t e = hipFuncSetAttribute((const void*)kern,                                       \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
        if (e != hipSuccess) {                                                                      \
            g_launch_reason = "hipFuncSetAttribute(max dynamic LDS) failed";                        \
            return e;                                                                               \
        }                                                                                           \
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), blk, lds, st, p, r,                          \
                           (const typename MF::elem*)Vt, (const typename MF::elem*)Cs, ldc, sigma,  \
                           kb_count, chunk, nchunks);                                               \
        return hipGetLastError();                                                                   \
    }
#define ABL_SPT(KBV, MTV, NSV)                                                                      \
    {                                                                                               \
        if (spt <= 2) ABL_GO(KBV, MTV, 2, NSV)                                                      \
        if (spt <= 4) ABL_GO(KBV, MTV, 4, NSV)                                                      \
        ABL_GO(KBV, MTV, 8, NSV)                                                                    \
    }
#define ABL_KB(KBV)                                                                                 \
    if (kb_count <= KBV) {                                                                          \
        if (NS == 1 && MT == 1) ABL_SPT(KBV, 1, 1)                                                  \
        if (NS == 1 && MT == 2) ABL_SPT(KBV, 2, 1)                                                  \
        if (NS == 1 && MT == 3) ABL_SPT(KBV, 3, 1)                                                  \
        if (NS == 1 && MT == 4) ABL_SPT(KBV, 4, 1)                                                  \
        if (NS == 4 && MT == 1) ABL_SPT(KBV, 1, 4)                                                  \
        ABL_SPT(KBV, 2, 4)                                                                          \
    }
    if constexpr (MF::K == 4) {
        ABL_KB(3)
        ABL_KB(5)
        ABL_KB(8)
        ABL_KB(11)
        ABL_KB(14)
        ABL_KB(18)
        ABL_KB(23)
    } else {
        ABL_KB(1)
        ABL_KB(2)
        ABL_KB(3)
        ABL_KB(4)
    }
#undef ABL_KB
#undef ABL_SPT
#undef ABL_GO
    return invalid("alpha-beta: no kernel variant for this K-block count");
}

// C (FP64, rows x cols) -> padded copy in the MFMA input type, row stride ld
template <typename T, typename TI>
__global__ void k_convert_pad(const TI* __restrict__ C, T* __restrict__ out, int64_t rows,
                              int64_t cols, int64_t ld)
{
    const int64_t total = rows * ld;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / ld, c = i - r * ld;
        out[i] = c < cols ? (T)(float)C[r * cols + c] : (T)0.f;
    }
}

template <typename MF>
static int64_t ab_lds_bytes(int kb_count, int64_t chunk)
{
    const int Kp = kb_count * MF::K;
    int64_t b = (chunk * (int64_t)sizeof(typename MF::lacc) + 15) / 16 * 16;
    b += ((int64_t)TileLayout<MF>::size(Kp) * sizeof(typename MF::elem) + 15) / 16 * 16;
    b += (int64_t)Kp * 4 + 64;
    return b;
}

template <typename MF, int KB, int MTV>
static hipError_t ab_launch_pf(const AbParams& p, const void* Vt, const double* C, double* sigma,
                               int kb_count, int64_t chunk, int nchunks, int nwaves, int pf,
                               hipStream_t st)
{
    const size_t lds = (size_t)ab_lds_bytes<MF>(kb_count, chunk);
    const int64_t items = p.Na * nchunks;
    const int64_t grid = (items + 7) / 8 * 8;
    dim3 blk(64 * nwaves);
#define AB_PF(PFV)                                                                                  \
    if (pf <= PFV) {                                                                                \
        auto kern = k_ab<MF, KB, MTV, PFV>;                                                         \
        hipError_t e = hipFuncSetAttribute((const void*)kern,                                       \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
        if (e != hipSuccess) {                                                                      \
            g_launch_reason = "hipFuncSetAttribute(max dynamic LDS) failed";                        \
            return e;                                                                               \
        }                                                                                           \
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), blk, lds, st, p,                             \
                           (const typename MF::elem*)Vt, C, sigma, kb_count, chunk, nchunks);       \
        return hipGetLastError();                                                                   \
    }
    AB_PF(4)
    AB_PF(8)
    AB_PF(12)
    AB_PF(16)
#undef AB_PF
    return invalid("alpha-beta: prefetch depth above 16");
}

template <typename MF>
static hipError_t ab_launch(const AbParams& p, const void* Vt, const double* C, double* sigma,
                            hipStream_t st)
{
    if (p.Na <= 0 || p.Nb <= 0 || p.sa <= 0 || p.M <= 0) return hipSuccess;
    const int kb_count = (p.sa + MF::K - 1) / MF::K;
    const int mtiles = p.Mp / 16;
    const int MT = mtiles > AB_MAX_WAVES ? 2 : 1;
    const int nwaves = (mtiles + MT - 1) / MT;
    if (nwaves > AB_MAX_WAVES) return invalid("alpha-beta: too many pair rows (norb too large)");
    const int64_t lds_cap = 160 * 1024 - 512;
    const int64_t fixed = ab_lds_bytes<MF>(kb_count, 0);
    int64_t chunk = (lds_cap - fixed) / (int64_t)sizeof(typename MF::lacc);
    if (chunk < 256) return invalid("alpha-beta: LDS too small for the sigma row chunk");
    int nchunks = (int)((p.Nb + chunk - 1) / chunk);
    chunk = (p.Nb + nchunks - 1) / nchunks;
    const int nth = 64 * nwaves;
    const int pf = (kb_count * MF::K * AB_TN + nth - 1) / nth;
    if (pf > 16) return invalid("alpha-beta: prefetch depth above 16");
    constexpr int KS = MF::K;
#define AB_KB(KBV, MTV)                                                                             \
    if (kb_count <= KBV && MT == MTV)                                                               \
        return ab_launch_pf<MF, KBV, MTV>(p, Vt, C, sigma, kb_count, chunk, nchunks, nwaves, pf, st);
    if constexpr (KS == 4) {
        // exact K-block counts of the common active spaces (n = 6..18) keep
        // the A fragments in registers without dead slots
        AB_KB(3, 1)
        AB_KB(5, 1)
        AB_KB(8, 1)
        AB_KB(11, 1)
        AB_KB(14, 1)
        AB_KB(18, 1)
        AB_KB(23, 1)
        AB_KB(28, 1)
        AB_KB(32, 1)
        AB_KB(8, 2)
        AB_KB(14, 2)
        AB_KB(18, 2)
        AB_KB(23, 2)
    } else {
        AB_KB(1, 1)
        AB_KB(2, 1)
        AB_KB(3, 1)
        AB_KB(4, 1)
        AB_KB(2, 2)
        AB_KB(3, 2)
        AB_KB(4, 2)
    }
#undef AB_KB
    return invalid("alpha-beta: no kernel variant for this K-block count");
}

hipError_t launch_ab_f64(const AbParams& p, const double* Vt, const double* C, double* sigma,
                         hipStream_t st)
{
    return ab_launch<MfmaF64>(p, Vt, C, sigma, st);
}

hipError_t launch_ab_lowp(const AbParams& p, const AbReduce& r, int prec, const void* Vt, const void* Cs,
                          int64_t ldc, float* sigma, hipStream_t st)
{
    if (prec == 1) return abl_launch<MfmaF32, float>(p, r, Vt, Cs, ldc, sigma, st);
    if (prec == 2) return abl_launch<MfmaBF16, float>(p, r, Vt, Cs, ldc, sigma, st);
    return invalid("alpha-beta: unknown precision");
}

hipError_t launch_ab_lowp(const AbParams& p, const AbReduce& r, int prec, const void* Vt, const void* Cs,
                          int64_t ldc, double* sigma, hipStream_t st)
{
    if (prec == 1) return abl_launch<MfmaF32, double>(p, r, Vt, Cs, ldc, sigma, st);
    if (prec == 2) return abl_launch<MfmaBF16, double>(p, r, Vt, Cs, ldc, sigma, st);
    return invalid("alpha-beta: unknown precision");
}

int64_t lowp_ld(int prec, int64_t cols)
{
    const int64_t v = prec == 1 ? 4 : 8;  // elements per 16 bytes
    return (cols + v - 1) / v * v;
}

hipError_t launch_convert_lowp(int prec, const double* C, void* out, int64_t rows, int64_t cols,
                               int64_t ld, hipStream_t st)
{
    const int64_t total = rows * ld;
    if (total <= 0) return hipSuccess;
    int64_t g = (total + 255) / 256;
    if (g > 16384) g = 16384;
    if (prec == 1)
        hipLaunchKernelGGL((k_convert_pad<float, double>), dim3((unsigned)g), dim3(256), 0, st, C, (float*)out,
                           rows, cols, ld);
    else
        hipLaunchKernelGGL((k_convert_pad<__bf16, double>), dim3((unsigned)g), dim3(256), 0, st, C, (__bf16*)out,
                           rows, cols, ld);
    return hipGetLastError();
}

hipError_t launch_convert_lowp_f32in(int prec, const float* C, void* out, int64_t rows, int64_t cols, int64_t ld,
                                     hipStream_t st)
{
    const int64_t total = rows * ld;
    if (total <= 0) return hipSuccess;
    int64_t g = (total + 255) / 256;
    if (g > 16384) g = 16384;
    if (prec == 1)
        hipLaunchKernelGGL((k_convert_pad<float, float>), dim3((unsigned)g), dim3(256), 0, st, C, (float*)out,
                           rows, cols, ld);
    else
        hipLaunchKernelGGL((k_convert_pad<__bf16, float>), dim3((unsigned)g), dim3(256), 0, st, C, (__bf16*)out,
                           rows, cols, ld);
    return hipGetLastError();
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


}  // namespace casci
