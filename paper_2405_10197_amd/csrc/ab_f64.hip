// FP64 alpha-beta contraction of the sigma build (Sec. II.A.1) on FP64 MFMA,
// with an order-independent (bitwise reproducible) scatter.
//
// One workgroup owns one alpha string Ia and one chunk [lo, hi) of its sigma
// row, accumulated in LDS. For every tile of AB_TN beta strings Jb the rows
// C(J_e, tile) of Ia's single-substitution list are gathered into LDS, each
// wave multiplies one or two 16-row tiles of pair rows (16x16x4 FP64 MFMA,
// four 16-column sub-tiles as independent accumulator chains) and scatters
// its accumulator elements to sigma(Ia, E_rs Jb) through the tabulated
// targets tg[Jb][m].
//
// Reproducibility. The contributions to one sigma element arrive from
// different waves in an order the hardware does not fix, so a floating-point
// sum would differ from run to run in its last bits. The row is accumulated
// in 64-bit fixed point instead: every contribution x is rounded once to an
// integer multiple of u = 2^(ex-62) and added with an integer LDS atomic,
// which is associative, so the result does not depend on the order. The unit
// u comes from a bound B < 2^ex on every partial sum: a sigma element of row
// Ia receives at most s_b contributions (one per entry of the target's beta
// list), each |T(m, Jb)| <= max_m sum_e |A(m, e)| * max_e max_Jb |C(J_e, Jb)|,
// so B = s_b * amax * cmax and every partial sum stays below 2^62 < 2^63.
// The rounding error of an element is at most s_b * u / 2, i.e. about
// 2^-62 s_b B relative to the bound.
#include "ab_common.h"

namespace casci {

// rowmax[J] = max_c |C(J, c)| (one wave per row, a fixed reduction order)
__global__ __launch_bounds__(256) void k_row_absmax(const double* __restrict__ C, int64_t rows, int64_t cols,
                                                    double* __restrict__ out)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t r = (int64_t)blockIdx.x * 4 + wave; r < rows; r += (int64_t)gridDim.x * 4) {
        const double* row = C + r * cols;
        double m = 0.0;
        bool bad = false;
        for (int64_t c = lane; c < cols; c += 64) {
            const double a = fabs(row[c]);
            bad = bad || !(a <= 1.7976931348623157e308);  // NaN or Inf
            m = fmax(m, a);
        }
        for (int off = 32; off > 0; off >>= 1) {
            m = fmax(m, __shfl_xor(m, off));
            bad = bad || __shfl_xor((int)bad, off);
        }
        if (lane == 0) out[r] = bad ? __builtin_inf() : m;
    }
}

hipError_t launch_row_absmax(const double* C, int64_t rows, int64_t cols, double* out, hipStream_t st)
{
    if (rows <= 0) return hipSuccess;
    int64_t g = (rows + 3) / 4;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_row_absmax, dim3((unsigned)g), dim3(256), 0, st, C, rows, cols, out);
    return hipGetLastError();
}

// targets of the accumulator elements a lane owns in one AB_TN-column tile
template <int MT>
__device__ inline void ab_load_targets(const AbParams& p, int64_t j0, int wave, int nwaves, int lane,
                                       i4 (&dst)[MT][4])
{
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int m0 = (wave + mt * nwaves) * 16;
#pragma unroll
        for (int ns = 0; ns < 4; ++ns) {
            // unconditional load at a clamped address (an M tile past the last
            // computes nothing; a column past the last reads column 0 and its
            // accumulators are zero): the loads stay in flight across the tile
            const int64_t jc = j0 + ns * 16 + (lane & 15);
            const int64_t jcc = jc < p.Nb ? jc : 0;
            const int m0c = m0 < p.Mp ? m0 : 0;
            dst[mt][ns] = *reinterpret_cast<const i4*>(p.tg + jcc * p.Mp + m0c + 4 * (lane >> 4));
        }
    }
}

// fixed-point scatter-add of one 16x64 accumulator block into the LDS row chunk
// [lo, hi): all sixteen conversions first (independent, so they pipeline), then
// the integer adds; an element without a target in the chunk goes to the
// lane's absorbing slot after the chunk (never read), so no add is conditional
__device__ inline void ab_scatter_fixed(unsigned long long* sig, const d4 (&acc)[4], const i4 (&tgt)[4],
                                        int64_t lo, int64_t hi, double scale, int absorb)
{
    long long q[4][4];
    int off[4][4];
#pragma unroll
    for (int ns = 0; ns < 4; ++ns) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int32_t e = tgt[ns][v];
            const int64_t tgi = l1_index(e);
            const bool in = e != AB_NONE && tgi >= lo && tgi < hi;
            off[ns][v] = in ? (int)(tgi - lo) : absorb;
            q[ns][v] = __double2ll_rn((e >= 0 ? acc[ns][v] : -acc[ns][v]) * scale);
        }
    }
#pragma unroll
    for (int ns = 0; ns < 4; ++ns)
#pragma unroll
        for (int v = 0; v < 4; ++v) atomicAdd(&sig[off[ns][v]], (unsigned long long)q[ns][v]);
}

// EXACT: kb_count == KBMAX, known at compile time, so the K-block loop has
// no run-time guard (with one, every K block was a branch that cost register
// copies and an MFMA drain before the next)
template <int KBMAX, int MT, int PF, bool EXACT>
__global__ __launch_bounds__(64 * AB_MAX_WAVES) void k_ab(AbParams p, const double* __restrict__ Vt,
                                                          const double* __restrict__ C,
                                                          const double* __restrict__ rowmax,
                                                          double* __restrict__ sigma, int kb_count_arg,
                                                          int64_t chunk, int nchunks)
{
    using MF = MfmaF64;
    __shared__ double s_amax[AB_MAX_WAVES], s_cmax[AB_MAX_WAVES];
    extern __shared__ __align__(16) unsigned char smem[];
    const int kb_count = EXACT ? KBMAX : kb_count_arg;
    const int Kp = kb_count * MF::K;
    unsigned long long* sig = reinterpret_cast<unsigned long long*>(smem);
    double* Dt = reinterpret_cast<double*>(smem + (((chunk + 64) * 8 + 15) / 16) * 16);
    int* sJ = reinterpret_cast<int*>(Dt + ((TileLayout<MF>::size(Kp) * 8 + 15) / 16) * 2);

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

    // the row chunk and, after it, one absorbing slot per lane
    for (int64_t i = tid; i < hi - lo + 64; i += nth) sig[i] = 0ull;
    for (int i = tid; i < Kp; i += nth) sJ[i] = i < p.sa ? l1_index(p.la_j[ia * p.sa + i]) : 0;

    // A fragments (row lane%16 of each M tile carries pair row arow(lane%16))
    double afr[MT][KBMAX];
    double amax = 0.0;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int m0 = (wave + mt * nwaves) * 16;
        const int m = m0 + MF::arow(lane & 15);
        double rs = 0.0;
#pragma unroll
        for (int kb = 0; kb < KBMAX; ++kb) {
            const int e = kb * MF::K + (lane >> 4);
            double v = 0.0;
            if (kb < kb_count && e < p.sa && m < p.M) {
                const int32_t enc = p.la_j[ia * p.sa + e];
                const int pq = p.la_pq[ia * p.sa + e];
                v = Vt[(int64_t)((pq & 0xff) * p.n + (pq >> 8)) * p.Mp + m];
                if (l1_sign(enc) < 0) v = -v;
            }
            afr[mt][kb] = v;
            rs += fabs(v);
        }
        // sum over the four lanes holding the same pair row, then the largest row
        rs += __shfl_xor(rs, 16);
        rs += __shfl_xor(rs, 32);
        amax = fmax(amax, rs);
    }
    double cmax = 0.0;
    for (int i = tid; i < p.sa; i += nth) cmax = fmax(cmax, rowmax[l1_index(p.la_j[ia * p.sa + i])]);
    for (int off = 1; off < 64; off <<= 1) {
        amax = fmax(amax, __shfl_xor(amax, off));
        cmax = fmax(cmax, __shfl_xor(cmax, off));
    }
    if (lane == 0) {
        s_amax[wave] = amax;
        s_cmax[wave] = cmax;
    }
    __syncthreads();
    amax = 0.0;
    cmax = 0.0;
    for (int w = 0; w < nwaves; ++w) {
        amax = fmax(amax, s_amax[w]);
        cmax = fmax(cmax, s_cmax[w]);
    }
    // fixed-point unit: B = s_b amax cmax < 2^ex, scale = 2^(62-ex) (exact inverse)
    const double B = (double)p.sb * amax * cmax;
    double* srow = sigma + ia * p.Nb;
    if (!(B <= 1.7976931348623157e308)) {  // a non-finite input row: propagate NaN
        for (int64_t i = tid; i < hi - lo; i += nth) srow[lo + i] = __builtin_nan("");
        return;
    }
    int ex = 0;
    if (B > 0.0) (void)frexp(B, &ex);
    // unit 2^-se, se = 62 - ex (capped where the bound is so small that the scale
    // alone could leave the double range)
    const int se = 62 - ex > 1000 ? 1000 : 62 - ex;
    const double scale = ldexp(1.0, se);
    const double unit = ldexp(1.0, -se);

    const int tile_elems = Kp * AB_TN;
    // A thread's tile elements are the same (list row, column) in every tile:
    // their rows are read from LDS once. The loads are unconditional at clamped
    // addresses, so the compiler's wait counts leave them in flight: padded
    // list rows meet zero A fragments, and columns past the last are stored to
    // LDS as zeros (their clamped targets are real ones and must receive 0).
    // (element idx = tid + i nth of a tile is list row idx / 64 = wave + i nwaves
    // and column idx % 64 = lane, as nth is a multiple of 64)
    static_assert(AB_TN == 64, "one column per lane");
    int rowJ[PF];
#pragma unroll
    for (int i = 0; i < PF; ++i) {
        const int k = wave + i * nwaves;
        rowJ[i] = k < p.sa ? sJ[k] : 0;
    }
    double pf[PF];
    auto load_tile = [&](int64_t j0) {
        const int64_t col = j0 + lane < p.Nb ? j0 + lane : 0;
#pragma unroll
        for (int i = 0; i < PF; ++i) pf[i] = C[(int64_t)rowJ[i] * p.Nb + col];
    };
    auto store_tile = [&](int64_t j0) {
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int idx = tid + i * nth;
            if (idx < tile_elems) {
                const int k = idx / AB_TN, c = idx - k * AB_TN;
                Dt[TileLayout<MF>::at(k, c, Kp)] = j0 + c < p.Nb ? pf[i] : 0.0;
            }
        }
    };
    const int absorb = (int)(hi - lo) + lane;
    // One tile: this tile's targets (their latency hides behind the FP64 MFMA
    // chain; a second register set for them would spill the A fragments) and
    // the next tile's D elements are issued first; past the last tile the loads
    // read the last tile again (unused).
    load_tile(0);
    store_tile(0);
    __syncthreads();
    for (int64_t j0 = 0; j0 < p.Nb; j0 += AB_TN) {
        const bool more = j0 + AB_TN < p.Nb;
        const int64_t jn = more ? j0 + AB_TN : j0;
        i4 tc[MT][4];
        ab_load_targets<MT>(p, j0, wave, nwaves, lane, tc);
        // keep the target loads ahead of the D loads: waiting for the targets
        // before the adds then leaves the D loads in flight
        __builtin_amdgcn_sched_barrier(0);
        load_tile(jn);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int mtile = wave + mt * nwaves;
            if (mtile * 16 >= p.Mp) continue;
            d4 acc[4];
#pragma unroll
            for (int ns = 0; ns < 4; ++ns)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[ns][v] = 0;
#pragma unroll
            for (int kb = 0; kb < KBMAX; ++kb) {
                if (kb < kb_count) {
#pragma unroll
                    for (int ns = 0; ns < 4; ++ns) {
                        const int c = ns * 16 + (lane & 15);
                        const double b = Dt[TileLayout<MF>::at(kb * MF::K + (lane >> 4), c, Kp)];
                        acc[ns] = MF::mma(afr[mt][kb], b, acc[ns]);
                    }
                }
            }
            ab_scatter_fixed(sig, acc, tc[mt], lo, hi, scale, absorb);
        }
        __syncthreads();
        if (more) store_tile(jn);
        __syncthreads();
    }
    if (p.overwrite)
        for (int64_t i = tid; i < hi - lo; i += nth) srow[lo + i] = (double)(long long)sig[i] * unit;
    else
        for (int64_t i = tid; i < hi - lo; i += nth) srow[lo + i] += (double)(long long)sig[i] * unit;
}

static int64_t ab_lds_bytes(int kb_count, int64_t chunk)
{
    const int Kp = kb_count * MfmaF64::K;
    int64_t b = ((chunk + 64) * 8 + 15) / 16 * 16;
    b += ((int64_t)TileLayout<MfmaF64>::size(Kp) * 8 + 15) / 16 * 16;
    b += (int64_t)Kp * 4 + 64;
    return b;
}

template <int KB, int MTV>
static hipError_t ab_launch_pf(const AbParams& p, const double* Vt, const double* C, const double* rowmax,
                               double* sigma, int kb_count, int64_t chunk, int nchunks, int nwaves, int pf,
                               hipStream_t st)
{
    const size_t lds = (size_t)ab_lds_bytes(kb_count, chunk);
    const int64_t items = p.Na * nchunks;
    const int64_t grid = (items + 7) / 8 * 8;
    dim3 blk(64 * nwaves);
#define AB_PF(PFV)                                                                                  \
    if (pf <= PFV) {                                                                                \
        auto kern = kb_count == KB ? k_ab<KB, MTV, PFV, true> : k_ab<KB, MTV, PFV, false>;          \
        hipError_t e = hipFuncSetAttribute((const void*)kern,                                       \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
        if (e != hipSuccess) {                                                                      \
            set_launch_reason("hipFuncSetAttribute(max dynamic LDS) failed");                       \
            return e;                                                                               \
        }                                                                                           \
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), blk, lds, st, p, Vt, C, rowmax, sigma,       \
                           kb_count, chunk, nchunks);                                               \
        return hipGetLastError();                                                                   \
    }
    AB_PF(4)
    AB_PF(8)
    AB_PF(12)
    AB_PF(16)
#undef AB_PF
    return ab_invalid("alpha-beta: prefetch depth above 16");
}

hipError_t launch_ab_f64(const AbParams& p, const double* Vt, const double* C, const double* rowmax,
                         double* sigma, hipStream_t st, int layout)
{
    if (p.Na <= 0 || p.Nb <= 0 || p.sa <= 0 || p.M <= 0) return hipSuccess;
    if (!rowmax) return ab_invalid("alpha-beta: row maxima of C missing");
    const int kb_count = (p.sa + MfmaF64::K - 1) / MfmaF64::K;
    const int mtiles = p.Mp / 16;
    // layout: 0 = default (one M tile per wave, two above AB_MAX_WAVES tiles;
    // the sigma row in as few LDS chunks as fit), else 10 MT + split with MT M
    // tiles per wave and split times the fewest chunks. Every layout gives the
    // same bits (integer sums), only the speed differs.
    const int lmt = layout / 10, lsplit = layout % 10;
    if (layout != 0 && (lmt < 1 || lmt > 2 || lsplit < 1 || lsplit > 4))
        return ab_invalid("alpha-beta: FP64 layout code must be 0 or 10 MT + split, MT 1..2, split 1..4");
    const int MT = layout != 0 ? lmt : (mtiles > AB_MAX_WAVES ? 2 : 1);
    const int nwaves = (mtiles + MT - 1) / MT;
    if (nwaves > AB_MAX_WAVES) return ab_invalid("alpha-beta: too many pair rows (norb too large)");
    // LDS: the static per-wave maxima plus the dynamic row chunk, D tile and row indices
    const int64_t lds_cap = 160 * 1024 - 512 - 2 * AB_MAX_WAVES * 8;
    const int64_t fixed = ab_lds_bytes(kb_count, 0);
    int64_t chunk = (lds_cap - fixed) / 8;
    if (chunk < 256) return ab_invalid("alpha-beta: LDS too small for the sigma row chunk");
    int nchunks = (int)((p.Nb + chunk - 1) / chunk) * (layout != 0 ? lsplit : 1);
    if (nchunks > p.Nb) nchunks = (int)p.Nb;
    chunk = (p.Nb + nchunks - 1) / nchunks;
    const int nth = 64 * nwaves;
    const int pf = (kb_count * MfmaF64::K * AB_TN + nth - 1) / nth;
    if (pf > 16) return ab_invalid("alpha-beta: prefetch depth above 16");
#define AB_KB(KBV, MTV)                                                                             \
    if (kb_count <= KBV && MT == MTV)                                                               \
        return ab_launch_pf<KBV, MTV>(p, Vt, C, rowmax, sigma, kb_count, chunk, nchunks, nwaves, pf, st);
    // exact K-block counts of the common active spaces (n = 6..18) keep the A
    // fragments in registers without dead slots
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
#undef AB_KB
    return ab_invalid("alpha-beta: no kernel variant for this K-block count");
}

}  // namespace casci
