// One- and two-particle reduced density matrices of a CI vector (the
// quantities the methods built on the CASCI solve consume, Sec. II.A.1 and
// the orbital optimisation and perturbation theories that follow it).
//
// With the pair-excitation vectors D^s_pq(K) = <K| E^s_pq |C> (s = alpha,
// beta; one vector per ordered orbital pair) the matrices are inner products:
//   <C| E^s_pq |C>            = sum_K C(K) D^s_pq(K)
//   <C| E^s_pq E^t_ru |C>     = sum_K D^s_qp(K) D^t_ru(K)      (E_pq^+ = E_qp)
//   <C| a+_ps a+_rt a_ut a_qs |C> = <C| E^s_pq E^t_ru |C> - d_st d_qr <C| E^s_pu |C>
// so all of them come from one Gram matrix G = M M^T of the rows
// M = [D^alpha_(pq) ; D^beta_(pq) ; C], accumulated over blocks of alpha
// strings (a plain GEMM). D^alpha_pq(Ka, Kb) = s C(J, Kb) for the entry
// (p, q, J, s) of Ka's single-substitution list, D^beta_pq(Ka, Kb) =
// s C(Ka, J) for the entry of Kb's list, zero where E_pq vanishes on the string.
#include "internal.h"

namespace casci {

// position of (p, q) in the single-substitution list of string m (p occupied,
// q unoccupied or q = p), or -1 when E_pq vanishes on m: the list runs over
// the occupied p ascending and, for each, over (unoccupied orbitals) + {p}
// ascending
__device__ inline int list_pos(uint64_t m, int p, int q, int n, int ne)
{
    if (!((m >> p) & 1)) return -1;
    if (q != p && ((m >> q) & 1)) return -1;
    const uint64_t nmask = n >= 64 ? ~0ull : ((1ull << n) - 1);
    const uint64_t below_p = p == 0 ? 0ull : ((1ull << p) - 1);
    const uint64_t below_q = q == 0 ? 0ull : ((1ull << q) - 1);
    return __popcll(m & below_p) * (n - ne + 1) + __popcll(~m & nmask & below_q) + (p < q ? 1 : 0);
}

// M[r][t] for the determinants t = (Ka - a0) * Nb + Kb of the block of alpha strings
// [a0, a0 + nblk): rows r < n^2 alpha pairs, n^2 <= r < 2 n^2 beta pairs, r = 2 n^2 C
__global__ __launch_bounds__(256) void k_rdm_fill(const double* __restrict__ C, int64_t a0, int64_t nblk,
                                                  int64_t Nb, int n, int na, int nb, const uint64_t* __restrict__ astr,
                                                  const uint64_t* __restrict__ bstr, const int32_t* __restrict__ la_j,
                                                  int sa, const int32_t* __restrict__ lb_j, int sb,
                                                  double* __restrict__ M, int64_t ldm)
{
    const int64_t total = nblk * Nb;
    const int n2 = n * n;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ka = a0 + t / Nb, kb = t % Nb;
        const uint64_t ma = astr[ka], mb = bstr[kb];
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) {
                double va = 0.0, vb = 0.0;
                const int pa = na > 0 ? list_pos(ma, p, q, n, na) : -1;
                if (pa >= 0) {
                    const int32_t e = la_j[ka * sa + pa];
                    const double c = C[(int64_t)l1_index(e) * Nb + kb];
                    va = l1_sign(e) > 0 ? c : -c;
                }
                const int pb = nb > 0 ? list_pos(mb, p, q, n, nb) : -1;
                if (pb >= 0) {
                    const int32_t e = lb_j[kb * sb + pb];
                    const double c = C[ka * Nb + l1_index(e)];
                    vb = l1_sign(e) > 0 ? c : -c;
                }
                M[(int64_t)(p * n + q) * ldm + t] = va;
                M[(int64_t)(n2 + p * n + q) * ldm + t] = vb;
            }
        M[(int64_t)(2 * n2) * ldm + t] = C[ka * Nb + kb];
    }
}

hipError_t launch_rdm_fill(const double* C, int64_t a0, int64_t nblk, int64_t Nb, int n, int na, int nb,
                           const uint64_t* astr, const uint64_t* bstr, const int32_t* la_j, int sa,
                           const int32_t* lb_j, int sb, double* M, int64_t ldm, hipStream_t st)
{
    const int64_t total = nblk * Nb;
    if (total <= 0) return hipSuccess;
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_rdm_fill, dim3((unsigned)g), dim3(256), 0, st, C, a0, nblk, Nb, n, na, nb, astr, bstr,
                       la_j, sa, lb_j, sb, M, ldm);
    return hipGetLastError();
}

// G (R x R, column-major, R = 2 n^2 + 1) -> g1[2][n][n], g2[3][n^4] (g2 may be null):
//   g1[s][p][q] = G[C row][s n^2 + p n + q]
//   g2[k][p][q][r][u] = G[(s, q p)][(t, r u)] - d_st d_qr g1[s][p][u], (s, t) = (a,a), (a,b), (b,b)
__global__ __launch_bounds__(256) void k_rdm_assemble(const double* __restrict__ G, int n, double* __restrict__ g1,
                                                      double* __restrict__ g2)
{
    const int n2 = n * n;
    const int64_t n4 = (int64_t)n2 * n2;
    const int64_t R = 2 * n2 + 1;
    const int64_t crow = 2 * n2;
    const int64_t total = 2 * n2 + (g2 ? 3 * n4 : 0);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i < 2 * n2) {
            g1[i] = G[i * R + crow];  // column i, row of C (G is symmetric)
            continue;
        }
        const int64_t j = i - 2 * n2;
        const int k = (int)(j / n4);
        int64_t x = j - (int64_t)k * n4;
        const int u = (int)(x % n);
        x /= n;
        const int r = (int)(x % n);
        x /= n;
        const int q = (int)(x % n);
        const int p = (int)(x / n);
        const int s = k == 2 ? 1 : 0, t = k == 0 ? 0 : 1;
        const int64_t row = (int64_t)s * n2 + q * n + p, colm = (int64_t)t * n2 + r * n + u;
        double v = G[colm * R + row];
        if (s == t && q == r) v -= G[((int64_t)s * n2 + p * n + u) * R + crow];
        g2[j] = v;
    }
}

hipError_t launch_rdm_assemble(const double* G, int n, double* g1, double* g2, hipStream_t st)
{
    const int64_t n2 = (int64_t)n * n;
    const int64_t total = 2 * n2 + (g2 ? 3 * n2 * n2 : 0);
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_rdm_assemble, dim3((unsigned)g), dim3(256), 0, st, G, n, g1, g2);
    return hipGetLastError();
}

// spin sums: gamma = g1[a] + g1[b]; Gamma_pqru = aa + bb + ab_pqru + ab_rupq
__global__ __launch_bounds__(256) void k_rdm_spin_free(const double* __restrict__ g1, const double* __restrict__ g2,
                                                       int n, double* __restrict__ gam, double* __restrict__ Gam)
{
    const int64_t n2 = (int64_t)n * n, n4 = n2 * n2;
    const int64_t total = n2 + (Gam ? n4 : 0);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i < n2) {
            gam[i] = g1[i] + g1[n2 + i];
            continue;
        }
        const int64_t j = i - n2;
        const int64_t pq = j / n2, ru = j % n2;
        Gam[j] = g2[j] + g2[2 * n4 + j] + g2[n4 + j] + g2[n4 + ru * n2 + pq];
    }
}

hipError_t launch_rdm_spin_free(const double* g1, const double* g2, int n, double* gam, double* Gam, hipStream_t st)
{
    const int64_t n2 = (int64_t)n * n;
    const int64_t total = n2 + (Gam ? n2 * n2 : 0);
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_rdm_spin_free, dim3((unsigned)g), dim3(256), 0, st, g1, g2, n, gam, Gam);
    return hipGetLastError();
}

}  // namespace casci
