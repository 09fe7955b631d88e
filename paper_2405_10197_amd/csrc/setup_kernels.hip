// Setup kernels of the string-based CASCI path (Sec. II.A.1 of the paper):
// string enumeration with gap-free addresses, single-substitution lists, the
// same-spin operator F and the determinant diagonal H_II.
//
// Strings are 64-bit masks (bit p = orbital p, Sec. III.C). The address of a
// string with occupied orbitals p_1 < p_2 < ... < p_k is
// sum_i binom(p_i, i) (1-based i): the rank of the mask among all k-subsets
// in ascending integer order. It is gap-free and needs no hash table.
#include "internal.h"

#include <algorithm>
#include <climits>

namespace casci {

__device__ inline int64_t rank_of(uint64_t mask, const int64_t* binom, int ld)
{
    int64_t r = 0;
    int k = 1;
    while (mask) {
        int p = __builtin_ctzll(mask);
        r += binom[p * ld + k];
        ++k;
        mask &= mask - 1;
    }
    return r;
}

__global__ void k_build_strings(int n, int ne, int64_t N, const int64_t* __restrict__ binom,
                                uint64_t* __restrict__ out)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N) return;
    const int ld = n + 1;
    int64_t r = idx;
    uint64_t mask = 0;
    int p = n - 1;
    for (int k = ne; k >= 1; --k) {
        // largest p with binom(p, k) <= r (binom(p,k) = 0 for p < k)
        while (binom[p * ld + k] > r) --p;
        mask |= 1ull << p;
        r -= binom[p * ld + k];
        --p;
    }
    out[idx] = mask;
}

// For string I: entries (p, q) with p occupied ascending and, for each p,
// q in (unoccupied U {p}) ascending; J = I - p + q and
// sign = <I| a+_p a_q |J> = (-1)^(occupied orbitals strictly between p and q).
__global__ void k_single_lists(int n, int ne, int64_t N, const uint64_t* __restrict__ strs,
                               const int64_t* __restrict__ binom, int s, int32_t* __restrict__ lj,
                               uint16_t* __restrict__ lpq)
{
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= N) return;
    const int ld = n + 1;
    const uint64_t mI = strs[I];
    int64_t e = I * (int64_t)s;
    for (int p = 0; p < n; ++p) {
        if (!((mI >> p) & 1)) continue;
        for (int q = 0; q < n; ++q) {
            if (q != p && ((mI >> q) & 1)) continue;
            uint64_t mJ = (mI & ~(1ull << p)) | (1ull << q);
            int sign = (__popcll(mI & between_mask(p, q)) & 1) ? -1 : 1;
            int32_t J = (int32_t)rank_of(mJ, binom, ld);
            lj[e] = l1_encode(J, sign);
            lpq[e] = (uint16_t)(p | (q << 8));
            ++e;
        }
    }
}

__device__ inline double eri4(const double* eri, int n, int p, int q, int r, int s)
{
    return eri[((int64_t)(p * n + q) * n + r) * n + s];
}

// Row I of the same-spin operator F = H of the (ne, 0) system without the
// scalar term (Slater-Condon rules for one spin; <pq||rs> = (pr|qs)-(ps|qr)).
// Entry order: diagonal, singles (p in I ascending, q not in I ascending),
// doubles (p1<p2 in I, q1<q2 not in I, lexicographic).
__global__ void k_same_spin_operator(int n, int ne, int64_t N, const uint64_t* __restrict__ strs,
                                     const int64_t* __restrict__ binom,
                                     const double* __restrict__ h, const double* __restrict__ eri,
                                     int r, int32_t* __restrict__ col, double* __restrict__ val)
{
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= N) return;
    const int ld = n + 1;
    const uint64_t mI = strs[I];
    int64_t e = I * (int64_t)r;

    // diagonal: sum_p h_pp + 1/2 sum_{p,q in I} [(pp|qq) - (pq|qp)]
    double d = 0.0;
    for (int p = 0; p < n; ++p) {
        if (!((mI >> p) & 1)) continue;
        d += h[p * n + p];
        for (int q = 0; q < n; ++q)
            if ((mI >> q) & 1) d += 0.5 * (eri4(eri, n, p, p, q, q) - eri4(eri, n, p, q, q, p));
    }
    col[e] = (int32_t)I;
    val[e] = d;
    ++e;

    // singles: I has p, J has q instead
    for (int p = 0; p < n; ++p) {
        if (!((mI >> p) & 1)) continue;
        for (int q = 0; q < n; ++q) {
            if ((mI >> q) & 1) continue;
            uint64_t mJ = (mI & ~(1ull << p)) | (1ull << q);
            double v = h[p * n + q];
            for (int t = 0; t < n; ++t)
                if (t != p && ((mI >> t) & 1))
                    v += eri4(eri, n, p, q, t, t) - eri4(eri, n, p, t, t, q);
            int sign = (__popcll(mI & between_mask(p, q)) & 1) ? -1 : 1;
            col[e] = (int32_t)rank_of(mJ, binom, ld);
            val[e] = sign * v;
            ++e;
        }
    }

    // doubles: I has p1<p2, J has q1<q2 instead;
    // value = Gamma * [(p1 q1|p2 q2) - (p1 q2|p2 q1)],
    // Gamma = <I| a+_p1 a+_p2 a_q2 a_q1 |J> accumulated operator by operator.
    for (int p1 = 0; p1 < n; ++p1) {
        if (!((mI >> p1) & 1)) continue;
        for (int p2 = p1 + 1; p2 < n; ++p2) {
            if (!((mI >> p2) & 1)) continue;
            for (int q1 = 0; q1 < n; ++q1) {
                if ((mI >> q1) & 1) continue;
                for (int q2 = q1 + 1; q2 < n; ++q2) {
                    if ((mI >> q2) & 1) continue;
                    uint64_t mJ = (mI & ~(1ull << p1) & ~(1ull << p2)) | (1ull << q1) | (1ull << q2);
                    uint64_t dd = mJ;
                    int par = __popcll(dd & ((1ull << q1) - 1));
                    dd &= ~(1ull << q1);
                    par += __popcll(dd & ((1ull << q2) - 1));
                    dd &= ~(1ull << q2);
                    par += __popcll(dd & ((1ull << p2) - 1));
                    dd |= 1ull << p2;
                    par += __popcll(dd & ((1ull << p1) - 1));
                    double v = eri4(eri, n, p1, q1, p2, q2) - eri4(eri, n, p1, q2, p2, q1);
                    col[e] = (int32_t)rank_of(mJ, binom, ld);
                    val[e] = (par & 1) ? -v : v;
                    ++e;
                }
            }
        }
    }
}

// H_II = F_a(Ia,Ia) + F_b(Ib,Ib) + sum_{p in Ia, q in Ib} (pp|qq) + shift
//        + lambda * [S^2]_II,  [S^2]_II = Ms^2 + Ms + nb - |Ia & Ib|
__global__ void k_diagonal(int n, int64_t Na, int64_t Nb, const uint64_t* __restrict__ astr,
                           const uint64_t* __restrict__ bstr, const double* __restrict__ fa, int ra,
                           const double* __restrict__ fb, int rb, const double* __restrict__ jpq,
                           double shift, double lambda_s2, double* __restrict__ out)
{
    extern __shared__ double sj[];
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) sj[t] = jpq[t];
    __syncthreads();
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < Na * Nb;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ia = x / Nb, ib = x - ia * Nb;
        const uint64_t a = astr[ia], b = bstr[ib];
        double v = fa[ia * ra] + fb[ib * rb] + shift;
        for (uint64_t aa = a; aa; aa &= aa - 1) {
            int p = __builtin_ctzll(aa);
            for (uint64_t bb = b; bb; bb &= bb - 1) v += sj[p * n + __builtin_ctzll(bb)];
        }
        if (lambda_s2 != 0.0) {
            int na = __popcll(a), nb = __popcll(b);
            double ms = 0.5 * (na - nb);
            v += lambda_s2 * (ms * ms + ms + nb - __popcll(a & b));
        }
        out[x] = v;
    }
}

static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_build_strings(int n, int ne, int64_t N, const int64_t* binom, uint64_t* out,
                                hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_build_strings, dim3(nblk(N, 256)), dim3(256), 0, st, n, ne, N, binom, out);
    return hipGetLastError();
}

hipError_t launch_single_lists(int n, int ne, int64_t N, const uint64_t* strs, const int64_t* binom,
                               int s, int32_t* lj, uint16_t* lpq, hipStream_t st)
{
    if (N <= 0 || s <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_single_lists, dim3(nblk(N, 128)), dim3(128), 0, st, n, ne, N, strs, binom, s,
                       lj, lpq);
    return hipGetLastError();
}

hipError_t launch_same_spin_operator(int n, int ne, int64_t N, const uint64_t* strs,
                                     const int64_t* binom, const double* h, const double* eri,
                                     int r, int32_t* col, double* val, hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_same_spin_operator, dim3(nblk(N, 64)), dim3(64), 0, st, n, ne, N, strs,
                       binom, h, eri, r, col, val);
    return hipGetLastError();
}

// Entries 1..r-1 of every operator row put in ascending column order (the
// diagonal stays at entry 0): one workgroup per row, bitonic sort of the
// (column, value) pairs in LDS, padded to P = 2^k >= r - 1 with columns
// INT32_MAX. Columns within a row are distinct, so the order is unique.
__global__ __launch_bounds__(256) void k_sort_ss_rows(int64_t N, int r, int P, int32_t* __restrict__ col,
                                                      double* __restrict__ val)
{
    extern __shared__ __align__(16) unsigned char sm[];
    double* sv = reinterpret_cast<double*>(sm);
    int32_t* sc = reinterpret_cast<int32_t*>(sv + P);
    const int m = r - 1;
    for (int64_t I = blockIdx.x; I < N; I += gridDim.x) {
        int32_t* c = col + I * r + 1;
        double* v = val + I * r + 1;
        for (int k = threadIdx.x; k < P; k += blockDim.x) {
            sc[k] = k < m ? c[k] : INT32_MAX;
            sv[k] = k < m ? v[k] : 0.0;
        }
        __syncthreads();
        for (int size = 2; size <= P; size <<= 1)
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int k = threadIdx.x; k < P; k += blockDim.x) {
                    const int l = k ^ stride;
                    if (l <= k) continue;
                    const bool up = (k & size) == 0;
                    const int32_t a = sc[k], b = sc[l];
                    if ((a > b) == up) {
                        sc[k] = b;
                        sc[l] = a;
                        const double t = sv[k];
                        sv[k] = sv[l];
                        sv[l] = t;
                    }
                }
                __syncthreads();
            }
        for (int k = threadIdx.x; k < m; k += blockDim.x) {
            c[k] = sc[k];
            v[k] = sv[k];
        }
        __syncthreads();
    }
}

int sort_ss_rows_max() { return 8192; }

hipError_t launch_sort_ss_rows(int64_t N, int r, int32_t* col, double* val, hipStream_t st)
{
    const int m = r - 1;
    if (N <= 0 || m <= 1) return hipSuccess;
    int P = 2;
    while (P < m) P <<= 1;
    if (P > sort_ss_rows_max()) {
        set_launch_reason("same-spin operator: rows too long to sort in LDS");
        return hipErrorInvalidValue;
    }
    const size_t lds = (size_t)P * 12;
    hipError_t e = hipFuncSetAttribute((const void*)k_sort_ss_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) {
        set_launch_reason("hipFuncSetAttribute(max dynamic LDS) failed");
        return e;
    }
    const unsigned g = (unsigned)std::min<int64_t>(N, 1 << 16);
    hipLaunchKernelGGL(k_sort_ss_rows, dim3(g), dim3(256), lds, st, N, r, P, col, val);
    return hipGetLastError();
}

hipError_t launch_diagonal(int n, int64_t Na, int64_t Nb, const uint64_t* astr,
                           const uint64_t* bstr, const double* fa, int ra, const double* fb, int rb,
                           const double* jpq, double shift, double lambda_s2, double* out,
                           hipStream_t st)
{
    int64_t nd = Na * Nb;
    if (nd <= 0) return hipSuccess;
    // capped grid (the launch size in work-items is 32-bit); the kernel strides
    const unsigned g = (unsigned)std::min<int64_t>((nd + 255) / 256, 1 << 20);
    hipLaunchKernelGGL(k_diagonal, dim3(g), dim3(256), sizeof(double) * n * n, st, n, Na,
                       Nb, astr, bstr, fa, ra, fb, rb, jpq, shift, lambda_s2, out);
    return hipGetLastError();
}

// H_IJ between the determinants I = dets[i], J = dets[j] of a small set (the
// start space of the eigensolver): diagonal from H_II; a same-spin
// difference from the same-spin operator row (plus, for a single
// substitution p <- q, the opposite-spin Coulomb part sign * sum_k (pq|kk));
// one substitution in each spin: sign_a sign_b (pq|rs); more: zero.
__global__ __launch_bounds__(256) void k_pspace_h(int n, int P, const int64_t* __restrict__ dets, int64_t Nb,
                                                  const uint64_t* __restrict__ astr,
                                                  const uint64_t* __restrict__ bstr,
                                                  const int32_t* __restrict__ fa_col,
                                                  const double* __restrict__ fa_val, int ra,
                                                  const int32_t* __restrict__ fb_col,
                                                  const double* __restrict__ fb_val, int rb,
                                                  const double* __restrict__ eri,
                                                  const double* __restrict__ diag, double* __restrict__ H)
{
    const int i = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P || i >= P) return;
    const int64_t I = dets[i], J = dets[j];
    const int64_t Ia = I / Nb, Ib = I - Ia * Nb, Ja = J / Nb, Jb = J - Ja * Nb;
    const uint64_t ia = astr[Ia], ib = bstr[Ib], ja = astr[Ja], jb = bstr[Jb];
    const int da = __popcll(ia ^ ja) / 2, db = __popcll(ib ^ jb) / 2;
    auto row_value = [&](const int32_t* col, const double* val, int r, int64_t row, int64_t c) {
        double x = 0.0;
        for (int e = 0; e < r; ++e)
            if (col[row * r + e] == (int32_t)c) x = val[row * r + e];
        return x;
    };
    // bra x = ket y - q + p: returns <x| a+_p a_q |y>
    auto single = [&](uint64_t x, uint64_t y, int& p, int& q) {
        p = __builtin_ctzll(x & ~y);
        q = __builtin_ctzll(y & ~x);
        return (__popcll(y & between_mask(p, q)) & 1) ? -1.0 : 1.0;
    };
    double v = 0.0;
    if (I == J) {
        v = diag[I];
    } else if (da + db > 2) {
        v = 0.0;
    } else if (db == 0) {
        v = row_value(fa_col, fa_val, ra, Ia, Ja);
        if (da == 1) {
            int p, q;
            const double sg = single(ia, ja, p, q);
            double c = 0.0;
            for (uint64_t bb = ib; bb; bb &= bb - 1) c += eri4(eri, n, p, q, __builtin_ctzll(bb), __builtin_ctzll(bb));
            v += sg * c;
        }
    } else if (da == 0) {
        v = row_value(fb_col, fb_val, rb, Ib, Jb);
        if (db == 1) {
            int p, q;
            const double sg = single(ib, jb, p, q);
            double c = 0.0;
            for (uint64_t aa = ia; aa; aa &= aa - 1) c += eri4(eri, n, p, q, __builtin_ctzll(aa), __builtin_ctzll(aa));
            v += sg * c;
        }
    } else {
        int p, q, r, t;
        const double sa = single(ia, ja, p, q);
        const double sb = single(ib, jb, r, t);
        v = sa * sb * eri4(eri, n, p, q, r, t);
    }
    H[(int64_t)i * P + j] = v;
}

hipError_t launch_pspace_h(int n, int P, const int64_t* dets, int64_t Nb, const uint64_t* astr,
                           const uint64_t* bstr, const int32_t* fa_col, const double* fa_val, int ra,
                           const int32_t* fb_col, const double* fb_val, int rb, const double* eri,
                           const double* diag, double* H, hipStream_t st)
{
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pspace_h, dim3((P + 255) / 256, P), dim3(256), 0, st, n, P, dets, Nb, astr, bstr, fa_col,
                       fa_val, ra, fb_col, fb_val, rb, eri, diag, H);
    return hipGetLastError();
}

// out[idx[i]] = v[i] (out zeroed by the caller)
__global__ void k_scatter_values(const int64_t* __restrict__ idx, const double* __restrict__ v, int P,
                                 double* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P) out[idx[i]] = v[i];
}

hipError_t launch_scatter_values(const int64_t* idx, const double* v, int P, double* out, hipStream_t st)
{
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_values, dim3((P + 255) / 256), dim3(256), 0, st, idx, v, P, out);
    return hipGetLastError();
}

}  // namespace casci
