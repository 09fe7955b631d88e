// Internal declarations shared by the host runtime and the HIP kernel files.
// Not part of the public ABI (include/casci.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <type_traits>

namespace casci {

// ---------------------------------------------------------------------------
// string bookkeeping shared by host and device code
// ---------------------------------------------------------------------------
// A single-substitution list entry is stored as two arrays: int32 J with the
// sign folded in (J >= 0: sign +1, stored ~J: sign -1) and uint16 pq = p | q<<8.
__host__ __device__ inline int32_t l1_encode(int32_t J, int sign) { return sign > 0 ? J : ~J; }
__host__ __device__ inline int32_t l1_index(int32_t v) { return v >= 0 ? v : ~v; }
__host__ __device__ inline int l1_sign(int32_t v) { return v >= 0 ? 1 : -1; }

// Tile pair (bi, bj), bi <= bj < nb, of index k in the row-by-row enumeration
// of the upper triangle (the pairs of the S + p S^T pass): row bi starts at
// s(bi) = bi nb - bi (bi - 1) / 2; the quadratic is inverted in floating point
// and the rounding settled with integer checks.
__host__ __device__ inline void tile_pair_of(int64_t k, int64_t nb, int64_t& bi, int64_t& bj)
{
    auto rs = [nb](int64_t b) { return b * nb - b * (b - 1) / 2; };
    const double q = (double)(2 * nb + 1);
    bi = (int64_t)((q - sqrt(q * q - 8.0 * (double)k)) * 0.5);
    bi = bi < 0 ? 0 : (bi > nb - 1 ? nb - 1 : bi);
    while (bi > 0 && rs(bi) > k) --bi;
    while (bi + 1 < nb && rs(bi + 1) <= k) ++bi;
    bj = bi + (k - rs(bi));
}

// bits strictly between orbitals a and b
__host__ __device__ inline uint64_t between_mask(int a, int b)
{
    int lo = a < b ? a : b, hi = a < b ? b : a;
    if (hi - lo < 2) return 0;
    uint64_t upto_hi = (hi >= 64) ? ~0ull : ((1ull << hi) - 1);
    uint64_t upto_lo1 = (lo + 1 >= 64) ? ~0ull : ((1ull << (lo + 1)) - 1);
    return upto_hi & ~upto_lo1;
}

// Reason of the last hipErrorInvalidValue returned by a launch wrapper of
// this library on the calling thread ("" if the error came from HIP itself).
const char* launch_reason();
void set_launch_reason(const char* why);

// ---------------------------------------------------------------------------
// launch wrappers (defined in the .hip files); all enqueue on `st`
// ---------------------------------------------------------------------------
// setup_kernels.hip
hipError_t launch_build_strings(int n, int ne, int64_t N, const int64_t* binom, uint64_t* out,
                                hipStream_t st);
hipError_t launch_single_lists(int n, int ne, int64_t N, const uint64_t* strs, const int64_t* binom,
                               int s, int32_t* lj, uint16_t* lpq, hipStream_t st);
// entries 1..r-1 of every row in ascending column order (diagonal first);
// rows longer than sort_ss_rows_max() + 1 entries are refused
int sort_ss_rows_max();
hipError_t launch_sort_ss_rows(int64_t N, int r, int32_t* col, double* val, hipStream_t st);
hipError_t launch_same_spin_operator(int n, int ne, int64_t N, const uint64_t* strs,
                                     const int64_t* binom, const double* h, const double* eri,
                                     int r, int32_t* col, double* val, hipStream_t st);
hipError_t launch_diagonal(int n, int64_t Na, int64_t Nb, const uint64_t* astr,
                           const uint64_t* bstr, const double* fa, int ra, const double* fb, int rb,
                           const double* jpq, double shift, double lambda_s2, double* out,
                           hipStream_t st);
// H_IJ over a small set of determinants dets[P] (row-major P x P)
hipError_t launch_pspace_h(int n, int P, const int64_t* dets, int64_t Nb, const uint64_t* astr,
                           const uint64_t* bstr, const int32_t* fa_col, const double* fa_val, int ra,
                           const int32_t* fb_col, const double* fb_val, int rb, const double* eri,
                           const double* diag, double* H, hipStream_t st);
// out[idx[i]] = v[i]
hipError_t launch_scatter_values(const int64_t* idx, const double* v, int P, double* out, hipStream_t st);

// sigma_kernels.hip, ab_*.hip
// A same-spin operator in row form: r entries per row, int32 columns and
// FP64 values; optional compact copies (16-bit columns when there are fewer
// than 65536 strings, FP32 values) that the gathers use when present.
// Row-blocked form of a same-spin operator (strip width code SS_BLOCKED): rows
// in blocks of 32 (16 where the unions of 32 rows are too wide); per block the
// sorted union of the columns its rows touch. The gather stages the union rows of X in LDS, a chunk at a time, and
// each row reads its operands there. Each row's entries 1..r-1 (ascending
// columns) are split by chunks of the union and stored per chunk as groups of
// four aligned to the entry index (group g holds entries 4g..4g+3): a slot
// whose entry lies outside the chunk holds value 0 and the chunk's first union
// row, so every group is read and added whole (built by ensure_ss_blocks in
// casci.cpp).
constexpr int SS_BLOCKED = 99;
constexpr int SS_BLK_W = 16;  // waves per workgroup; a block has SS_BLK_W or 2 SS_BLK_W rows
constexpr int SS_BLK_MAXCH = 127;  // union limit: SS_BLK_MAXCH chunks of SS_BLK_CH rows per block
// union rows per LDS chunk, and bytes per staged row (64 FP64 columns or
// 128 FP32 column pairs): 32 KB per chunk buffer
constexpr int SS_BLK_CH = 64, SS_BLK_ROWB = 512;
// one group: the byte offsets of the four operands' rows within the LDS chunk
// ((union position mod SS_BLK_CH) x SS_BLK_ROWB) and the four values
struct SsGroup {
    uint32_t off[4];
    double v[4];
};
// the same group with FP32 values, for the FP32-accumulating gather of the
// BF16 sigma build (32 bytes: one scalar load)
struct SsGroupF {
    uint32_t off[4];
    float v[4];
};
template <typename TA>
using SsGroupOf = typename std::conditional<std::is_same<TA, float>::value, SsGroupF, SsGroup>::type;
struct SsBlk {
    const uint16_t* uni;   // unions of all blocks, concatenated (string indices < 65536)
    const int4* binfo;     // per block {union offset, union size, group offsets offset, chunks}
    const uint16_t* goff;  // per block [rows][chunks + 1]: first group of each chunk, per row
    const int32_t* rbase;  // [N]: first group of each row
    const SsGroup* gs64;   // groups with FP64 values (FP64 input)
    const SsGroup* gs32;   // groups with values rounded to FP32 (FP32 input)
    const SsGroupF* gsf;   // the gs32 groups with FP32 values (FP32 input, FP32 accumulation)
    int ch;                // union rows per chunk (SS_BLK_CH)
    int rows;              // rows per block (SS_BLK_W or 2 SS_BLK_W)
    int64_t nblk;
};
struct SsOp {
    const int32_t* col;
    const double* val;
    const uint16_t* col16;  // may be null
    const float* val32;     // may be null
    int r;
    SsBlk blk = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0, 0};  // row-blocked form (blk.uni null: none)
};
// Y(I,:) = [acc ? Y(I,:) : 0] + sum_e val[I*r+e] X(col[I*r+e], :) + shift * X(I,:)
// (lpe: strip width code 16/32/64 lanes per entry, 128 = 64 lanes x 2 columns; 0 = 64).
// FP64 X and Y: FP64 values (16-bit columns when present).
hipError_t launch_ss_gather_f64(const SsOp& op, int64_t nrows, int64_t ncols, const double* X, double* Y,
                                double shift, int acc, hipStream_t st, int lpe = 0);
// FP32 copy of X with row stride ldx, FP64 Y (compact operator when present).
// acc32: the row-blocked width accumulates in FP32 (FP32 values, no
// conversions per entry); the BF16 build uses it, whose alpha-beta part has a
// rounding error far above that of FP32 sums. Other widths ignore it.
hipError_t launch_ss_gather_f32in(const SsOp& op, int64_t nrows, int64_t ncols, const float* X, int64_t ldx,
                                  double* Y, double shift, int acc, hipStream_t st, int lpe = 0,
                                  bool acc32 = false);
// FP32 X and Y (FP64 accumulation; compact operator when present)
hipError_t launch_ss_gather_f32(const SsOp& op, int64_t nrows, int64_t ncols, const float* X, float* Y,
                                double shift, int acc, hipStream_t st, int lpe = 0);
hipError_t launch_compact_op(const int32_t* col, const double* val, int64_t n, uint16_t* col16, float* val32,
                             hipStream_t st);
// S <- scale (S + p S^T) [+ T], S square n x n, in place (T may be null).
// nrm2 (may be null): per-workgroup sums of squares of the result, one per
// tile pair (sym_add_parts(n) of them), for launch_reduce_partials
hipError_t launch_sym_add(double* S, int64_t n, int p, double scale, hipStream_t st,
                          const double* T = nullptr, double* nrm2 = nullptr);
inline int64_t sym_add_parts(int64_t n)
{
    const int64_t nb = (n + 31) / 32;
    return nb * (nb + 1) / 2;
}
// out[o] = sum over k of work[o * nparts + k] in a fixed order, o < nout
hipError_t launch_reduce_partials(const double* work, int nout, int nparts, double* out, hipStream_t st);
// out[j][i] (+)= in[i][j], in: rows x cols
hipError_t launch_transpose_f64(const double* in, double* out, int64_t rows, int64_t cols, int acc,
                                double scale, hipStream_t st);
hipError_t launch_transpose_f32(const float* in, float* out, int64_t rows, int64_t cols, int acc,
                                hipStream_t st);

struct AbParams {
    int n, nb;            // orbitals, beta electrons
    int64_t Na, Nb;       // string counts
    int sa;               // alpha list length
    int M, Mp;            // pair rows (real, padded to 16)
    int full;             // 1: ordered pairs (r,s) r,s < n; 0: r <= s
    const int32_t* la_j;  // alpha single list
    const uint16_t* la_pq;
    const uint64_t* bstr;
    const int32_t* lb_j;  // beta single list (targets of the scatter)
    int sb;               // beta list length
    const uint16_t* pairs;// [Mp] r | s << 8
    const int32_t* tg;    // [Nb][Mp] scatter targets (launch_ab_targets)
    int overwrite;        // 1: sigma(Ia,:) = term; 0: sigma(Ia,:) += term
};
// tg[Jb][m] = E_{r_m s_m} Jb as a list entry (index, sign folded), INT32_MIN where it vanishes
hipError_t launch_ab_targets(const AbParams& p, int32_t* tg, hipStream_t st);
// Target-grouped scatter table of the low-precision alpha-beta kernel. For
// each 64-column tile of beta strings Jb, the contributions (m, Jb) -> Ib of
// that tile are grouped by target Ib; the groups, sorted by size (largest
// first), are packed 64 to a chunk (one group per lane), and the chunks are
// dealt to the W waves of the workgroup, longest first to the least loaded
// one. A tile's block of 16-byte segments holds, each section padded to 16
// bytes:
//   wb[W+1]           uint16: wave w reduces chunks wb[w] .. wb[w+1]-1
//   desc[nchunk]      uint32: first block | blocks << 20
//   tgt[nchunk*64]    uint16: target Ib of each lane's group (0xffff: none)
//   off[blocks*64*4]  uint16: T-tile offset (Jb_local * ldT + m) | sign << 15;
//                             block b, lane l holds the lane's contributions
//                             4b..4b+3 at [(b*64 + l)*4 + 0..3]; unused slots
//                             point to the zero slot 64 * ldT
// tinfo[t] = {first segment, nseg | nchunk << 20}. Targets fit 16 bits, so
// the table needs Nb < 65535.
struct AbReduce {
    const uint4* tab;
    const int2* tinfo;
    int max_nseg;  // largest tile block, in segments
    int ldT;       // row stride (floats) of the LDS T tile: Mp + 4
};
// waves per workgroup of the low-precision alpha-beta kernel for Mp pair rows
int abl_waves(int Mp);
// sigma(Ia, :) += alpha-beta term; Vt[pq][Mp] in the arithmetic's type
// (prec 1: float, FP32 MFMA; prec 2: bf16, BF16 MFMA; both accumulate in FP32)
// FP64: fixed-point (order-independent) accumulation; rowmax[Na] = max_c |C(J, c)|
// from launch_row_absmax bounds the partial sums. layout: 0 (default) or
// 10 MT + split (MT = 1, 2 M tiles per wave; the sigma row in split times the
// fewest LDS chunks, split 1..4); a layout without a kernel variant for this
// shape returns hipErrorInvalidValue. All layouts give the same bits.
hipError_t launch_ab_f64(const AbParams& p, const double* Vt, const double* C, const double* rowmax,
                         double* sigma, hipStream_t st, int layout = 0);
hipError_t launch_row_absmax(const double* C, int64_t rows, int64_t cols, double* out, hipStream_t st);
hipError_t launch_ab_lowp(const AbParams& p, const AbReduce& r, int prec, const void* Vt, const void* Cs,
                          int64_t ldc, double* sigma, hipStream_t st);
// same, for an FP32 sigma (FP32-storage builds)
hipError_t launch_ab_lowp(const AbParams& p, const AbReduce& r, int prec, const void* Vt, const void* Cs,
                          int64_t ldc, float* sigma, hipStream_t st);
// per-precision instances (ab_lowp_{f32,bf16}_{d,f}.hip)
hipError_t launch_ab_lowp_f32(const AbParams& p, const AbReduce& r, const void* Vt, const void* Cs, int64_t ldc,
                              double* sigma, hipStream_t st);
hipError_t launch_ab_lowp_f32(const AbParams& p, const AbReduce& r, const void* Vt, const void* Cs, int64_t ldc,
                              float* sigma, hipStream_t st);
hipError_t launch_ab_lowp_bf16(const AbParams& p, const AbReduce& r, const void* Vt, const void* Cs, int64_t ldc,
                               double* sigma, hipStream_t st);
hipError_t launch_ab_lowp_bf16(const AbParams& p, const AbReduce& r, const void* Vt, const void* Cs, int64_t ldc,
                               float* sigma, hipStream_t st);
// BF16 contraction with the scatter from the accumulators into a 32-bit
// fixed-point sigma row (ab_bf16_fixed.hip): symmetric pairs, Nb + 64 < 32768 and
// the row in LDS; tg16 from launch_tg16 (tg16_entries(Nb, Mp) entries)
bool ab_bf16_fixed_fits(int64_t Nb, int sa, int Mp);
int64_t tg16_entries(int64_t Nb, int Mp);
hipError_t launch_tg16(const int32_t* tg, int64_t Nb, int Mp, uint16_t* out, hipStream_t st);
hipError_t launch_ab_bf16_fixed(const AbParams& p, const void* Vt, const void* Cs, int64_t ldc, const double* rowmax,
                                const uint16_t* tg16, double* sigma, hipStream_t st);
hipError_t launch_ab_bf16_fixed(const AbParams& p, const void* Vt, const void* Cs, int64_t ldc, const double* rowmax,
                                const uint16_t* tg16, float* sigma, hipStream_t st);
// padded row stride of the low-precision copy of C, and the conversion itself
int64_t lowp_ld(int prec, int64_t cols);
hipError_t launch_convert_lowp(int prec, const double* C, void* out, int64_t rows, int64_t cols,
                               int64_t ld, hipStream_t st);
hipError_t launch_convert_lowp_f32in(int prec, const float* C, void* out, int64_t rows, int64_t cols, int64_t ld,
                                     hipStream_t st);
hipError_t launch_convert_f64_to_f32(const double* in, float* out, int64_t n, hipStream_t st);
hipError_t launch_convert_f32_to_f64(const float* in, double* out, int64_t n, hipStream_t st);
hipError_t launch_axpby_f64(double a, const double* x, double b, double* y, int64_t n, hipStream_t st);

// davidson_kernels.hip
// partial dots: out[i*nb+j] = sum_x A_i[x] B_j[x]; A_i = A + i*lda, B_j = B + j*ldb
hipError_t launch_block_dot(const double* A, int64_t lda, int na, const double* B, int64_t ldb,
                            int nb, int64_t len, double* work, double* out, hipStream_t st);
// Y_j = beta*Y_j + sum_i A_i coef[i*ldc + j], j < nc (coef on device)
hipError_t launch_combine(const double* A, int64_t lda, int na, const double* coef, int ldc, int nc,
                          double beta, double* Y, int64_t ldy, int64_t len, hipStream_t st);
// residual norms / Olsen dots for k roots:
// r = SX_k - th_k X_k; out[k*4+0] = |r|^2, [1] = x.(D-th)^-1 r, [2] = x.(D-th)^-1 x
hipError_t launch_residual(const double* X, const double* SX, int64_t ld, int k, const double* theta,
                           const double* diag, int64_t len, double* work, double* out,
                           hipStream_t st);
// t = -(D-th)^-1 r + eps (D-th)^-1 x  (eps = 0 for the diagonal preconditioner)
hipError_t launch_precondition(const double* X, const double* SX, double theta, double eps,
                               const double* diag, int64_t len, double* T, hipStream_t st);
hipError_t launch_scale(double* x, double a, int64_t n, hipStream_t st);
// out[0] = x_i and out[1] = i for the largest |x_i| (ties: lowest i); work holds
// 2 * 512 doubles of partials
hipError_t launch_absmax(const double* x, int64_t n, double* work, double* out, hipStream_t st);
// out[0..nblk) per-block minima and out[nblk..2 nblk) maxima of x[0..n)
// (nblk <= 512, returned in *nblk_out)
hipError_t launch_minmax(const double* x, int64_t n, double* out, int* nblk_out, hipStream_t st);
// hist[b] += number of entries in bin b = clamp(floor((x - lo) inv_w), 0, nbins - 1)
hipError_t launch_value_hist(const double* x, int64_t n, double lo, double inv_w, int nbins, unsigned* hist,
                             hipStream_t st);
// (index, value) of every entry in bins <= bmax, in any order, the first cap kept;
// *count (zeroed by the caller) ends as the number found
hipError_t launch_value_collect(const double* x, int64_t n, double lo, double inv_w, int nbins, int bmax,
                                unsigned long long* count, int64_t* idx, double* val, int64_t cap, hipStream_t st);

// rdm_kernels.hip (density matrices)
// rows [D^alpha_pq ; D^beta_pq ; C] (row stride ldm) of the determinants of alpha strings [a0, a0 + nblk)
hipError_t launch_rdm_fill(const double* C, int64_t a0, int64_t nblk, int64_t Nb, int n, int na, int nb,
                           const uint64_t* astr, const uint64_t* bstr, const int32_t* la_j, int sa,
                           const int32_t* lb_j, int sb, double* M, int64_t ldm, hipStream_t st);
// spin-resolved g1[2][n][n] and g2[3][n^4] (may be null) from the Gram matrix G (R = 2n^2+1, column-major)
hipError_t launch_rdm_assemble(const double* G, int n, double* g1, double* g2, hipStream_t st);
// spin sums gamma[n][n], Gamma[n^4] (may be null) of g1, g2
hipError_t launch_rdm_spin_free(const double* g1, const double* g2, int n, double* gam, double* Gam, hipStream_t st);

// mlp_kernels.hip (learned preconditioner)
constexpr int MLP_IN = 8, MLP_HIDDEN = 64;
constexpr int MLP_NPARAM = MLP_IN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN +
                           MLP_HIDDEN + 1;
struct MlpFeatArgs {
    const double* diag;
    const double* x;   // Ritz vector
    const double* sx;  // its sigma
    double theta, rnorm, dmin;
    const uint64_t* astr;
    const uint64_t* bstr;
    int64_t N, Nb;
    int n, na, nb;
};
hipError_t launch_mlp_correction(const MlpFeatArgs& a, const float* P, double* t, hipStream_t st);
hipError_t launch_mlp_collect(const MlpFeatArgs& a, const int64_t* idx, int m, const double* xstar,
                              double xsign, double dnorm_inv, float* F, float* T, hipStream_t st);
hipError_t launch_mlp_forward(const float* P, const float* X, int64_t N, float* Y, hipStream_t st);
// one gradient of the mean squared error over samples perm[begin, begin+count) of
// `total` (the loss is normalised by total); partial holds nblocks*(NPARAM+1) floats
hipError_t launch_mlp_grad(const float* P, const float* X, const float* T, const int32_t* perm,
                           int64_t begin, int64_t count, int64_t total, float* partial, int nblocks,
                           float* grad, double* sse, hipStream_t st);
hipError_t launch_adam(float* P, const float* g, float* m, float* v, float lr, int step, hipStream_t st);

}  // namespace casci
