// BF16 alpha-beta contraction (BF16 MFMA, FP32 accumulation) with the scatter
// done straight from the accumulator registers into a 32-bit fixed-point sigma
// row in LDS.
//
// Same contraction as the other alpha-beta kernels (ab_common.h): one
// workgroup owns one alpha string Ia and its whole sigma row; per tile of
// AB_TN beta strings Jb the rows C(J_e, tile) of Ia's list are gathered into
// one of two LDS buffers (the next tile's loads are in flight while the
// current one is multiplied), each wave multiplies its pair-row tiles with
// 16x16x32 BF16 MFMA, and every accumulator element T(m, Jb) is added to
// sigma(Ia, E_m Jb) with an integer LDS atomic. There is no T tile in LDS, no
// reduction table and one barrier per tile.
//
// Fixed point. Integer adds are associative, so the row does not depend on
// the order in which waves add (bitwise reproducible), which floating-point
// LDS atomics would not give. Every partial sum of a sigma element is bounded
// by B = s_b amax cmax (s_b contributions per element, one per entry of its
// beta list; |T(m, Jb)| <= max_m sum_e |A(m, e)| max_e max_Jb |C(J_e, Jb)|,
// with a 1% margin for the BF16 rounding of C); with B < 2^ex the unit is
// 2^(ex-30), so every partial sum stays below 2^30 < 2^31. The rounding of a
// contribution to the unit adds at most 2^-31 B, far below the BF16 rounding
// of the inputs (2^-9 relative).
//
// Targets: a 16-bit table in the order of the MFMA accumulator elements, one
// 8-byte load per lane and 16x16 block: entry [lane][v] of block (tile, M
// tile, sub-tile) is pair row 16 mt + 4 (lane / 16) + v and column
// 64 t + 16 ns + lane % 16; bits 0-14 = the target beta string, bit 15 =
// negative sign. Where E_m Jb vanishes (or the column is past the last) the
// entry names slot Nb + lane, one of 64 slots after the sigma row in LDS that
// absorb such contributions and are never read, so the kernel adds every
// element without a test. It needs Nb + 64 < 32768; the sigma row needs
// (Nb + 64) * 4 bytes of LDS (Nb <= 15296).
#include "ab_common.h"

namespace casci {

constexpr int ABF_WAVES = 12;  // 4 column groups x 3 pair-row groups

__global__ __launch_bounds__(256) void k_tg16(const int32_t* __restrict__ tg, int64_t Nb, int Mp, int64_t ntile,
                                              uint16_t* __restrict__ out)
{
    const int mtiles = Mp / 16;
    const int64_t total = ntile * mtiles * 4 * 256;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t blk = i / 256;
        const int w = (int)(i % 256);
        const int lane = w / 4, v = w % 4;
        const int ns = (int)(blk % 4);
        const int64_t rest = blk / 4;
        const int mt = (int)(rest % mtiles);
        const int64_t t = rest / mtiles;
        const int m = mt * 16 + 4 * (lane >> 4) + v;
        const int64_t jc = t * AB_TN + ns * 16 + (lane & 15);
        uint16_t val = (uint16_t)(Nb + lane);  // absorbing slot of this lane
        if (jc < Nb) {
            const int32_t e = tg[jc * Mp + m];
            if (e != AB_NONE) val = (uint16_t)((l1_index(e) & 0x7fff) | (e < 0 ? 0x8000 : 0));
        }
        out[i] = val;
    }
}

hipError_t launch_tg16(const int32_t* tg, int64_t Nb, int Mp, uint16_t* out, hipStream_t st)
{
    if (Nb <= 0) return hipSuccess;
    if (Nb + 64 > 0x7fff) return ab_invalid("alpha-beta: 16-bit targets need Nb + 64 < 32768 beta strings");
    if (Mp % 16 != 0) return ab_invalid("alpha-beta: pair rows not padded to 16");
    const int64_t ntile = (Nb + AB_TN - 1) / AB_TN;
    const int64_t total = ntile * (Mp / 16) * 4 * 256;
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_tg16, dim3((unsigned)g), dim3(256), 0, st, tg, Nb, Mp, ntile, out);
    return hipGetLastError();
}

int64_t tg16_entries(int64_t Nb, int Mp)
{
    return (Nb + AB_TN - 1) / AB_TN * (Mp / 16) * 4 * 256;
}

template <typename TO, int KBMAX, int MT>
__global__ __launch_bounds__(64 * ABF_WAVES) void k_ab_bf16(AbParams p, const __bf16* __restrict__ Vt,
                                                            const __bf16* __restrict__ Cs, int64_t ldc,
                                                            const double* __restrict__ rowmax,
                                                            const uint16_t* __restrict__ tg16,
                                                            TO* __restrict__ sigma, int kb_count)
{
    using MF = MfmaBF16;
    using vec_t = uint4;
    constexpr int VEC = 8;            // bf16 per 16-byte segment
    constexpr int SEGS = AB_TN / VEC; // segments per tile row
    __shared__ double s_amax[ABF_WAVES], s_cmax[ABF_WAVES];
    extern __shared__ __align__(16) unsigned char smem[];
    const int Kp = kb_count * MF::K;
    const int tsz = ((TileLayout<MF>::size(Kp) * 2 + 15) / 16) * 16;  // bytes of one D buffer
    // sigma row, then one slot per lane that absorbs the (zero) contributions of
    // entries without a target, so that every atomic add is unconditional
    unsigned* sig = reinterpret_cast<unsigned*>(smem);
    const int64_t nsig = ((p.Nb + 64) * 4 + 15) / 16 * 4;
    unsigned char* dbase = smem + nsig * 4;
    int* sJ = reinterpret_cast<int*>(dbase + 2 * tsz);

    const int64_t per_xcd = gridDim.x / 8;
    const int64_t ia = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (ia >= p.Na) return;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int ngrp = wave & 3, mgrp = wave >> 2;
    const int mtiles = p.Mp / 16;

    for (int64_t i = tid; i < p.Nb + 64; i += nth) sig[i] = 0u;
    for (int i = tid; i < Kp; i += nth) sJ[i] = i < p.sa ? l1_index(p.la_j[ia * p.sa + i]) : -1;

    // A fragments: row lane % 16 of M tile (mgrp * MT + mt), k = 32 kb + 8 (lane / 16) + q
    typename MF::frag afr[MT][KBMAX];
    double amax = 0.0;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int m = (mgrp * MT + mt) * 16 + (lane & 15);
        double rs = 0.0;
#pragma unroll
        for (int kb = 0; kb < KBMAX; ++kb) {
            typename MF::frag f;
            // unconditional loads at clamped indices (then masked): the loads of
            // a fragment are in flight together
            int32_t enc[8];
            int pqv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = kb * MF::K + (lane >> 4) * 8 + q;
                const int ec = e < p.sa ? e : p.sa - 1;
                enc[q] = p.la_j[ia * p.sa + ec];
                pqv[q] = p.la_pq[ia * p.sa + ec];
            }
            const int mc = m < p.M ? m : p.M - 1;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = kb * MF::K + (lane >> 4) * 8 + q;
                __bf16 v = Vt[(int64_t)((pqv[q] & 0xff) * p.n + (pqv[q] >> 8)) * p.Mp + mc];
                if (l1_sign(enc[q]) < 0) v = -v;
                if (!(kb < kb_count && e < p.sa && m < p.M)) v = (__bf16)0.0f;
                f[q] = v;
                rs += fabs((double)(float)v);
            }
            afr[mt][kb] = f;
        }
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
    for (int w = 0; w < nth / 64; ++w) {
        amax = fmax(amax, s_amax[w]);
        cmax = fmax(cmax, s_cmax[w]);
    }
    TO* srow = sigma + ia * p.Nb;
    const double B = (double)p.sb * amax * cmax * 1.01;
    int ex = 0;
    if (B > 0.0) (void)frexp(B, &ex);
    // unit 2^-se with se = 30 - ex; below 2^-96 the bound leaves room for the largest
    // FP32 scale (se = 126), above 2^156 the FP32 scale would underflow
    int se = 30 - ex;
    if (se > 126) se = 126;
    if (!(B <= 1.7976931348623157e308) || se < -126) {  // a non-finite (or far too large) row: NaN
        for (int64_t i = tid; i < p.Nb; i += nth) srow[i] = (TO)__builtin_nan("");
        return;
    }
    const float scale = ldexpf(1.0f, se);
    const double unit = ldexp(1.0, -se);

    const int nseg = Kp * SEGS;
    const int64_t ntiles = (p.Nb + AB_TN - 1) / AB_TN;
    constexpr int SPT = 2;  // segments per thread: Kp * 8 <= 2 * 768 for Kp <= 192
    // A thread's segments are the same (list row, 8 columns) in every tile: their
    // rows are read from LDS once. The loads are unconditional and their values
    // used as loaded, so that the compiler's wait counts leave the next tile's
    // loads in flight across the current tile's work: a padded list row (k >=
    // s_alpha) reads row 0 and meets zero A fragments, columns past the row
    // read its first columns and have no targets.
    int64_t rowoff[SPT];
    int segc[SPT];
    bool segok[SPT];  // (sJ is complete: the barrier after the row maxima follows its writes)
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
        const int sidx = tid + q * nth;
        const int k = sidx < nseg ? sidx / SEGS : 0;
        const int J = sidx < nseg ? sJ[k] : -1;
        segc[q] = (sidx - k * SEGS) * VEC;
        segok[q] = sidx < nseg && J >= 0;
        rowoff[q] = (int64_t)(J >= 0 ? J : 0) * ldc;
    }
    vec_t pf[SPT];
    auto issue = [&](int64_t tile) {
        const int64_t j0 = tile * AB_TN;
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int64_t col = j0 + segc[q];
            const bool ok = segok[q] && col < ldc;
            pf[q] = *reinterpret_cast<const vec_t*>(Cs + rowoff[q] + (ok ? col : 0));
        }
    };
    auto commit = [&](int buf) {
        __bf16* Dt = reinterpret_cast<__bf16*>(dbase + buf * tsz);
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int sidx = tid + q * nth;
            if (sidx < nseg) {
                const int k = sidx / SEGS, sg = sidx - k * SEGS;
                const __bf16* ve = reinterpret_cast<const __bf16*>(&pf[q]);
#pragma unroll
                for (int e = 0; e < VEC; ++e) Dt[TileLayout<MF>::at(k, sg * VEC + e, Kp)] = ve[e];
            }
        }
    };
    // this lane's targets of one tile: 4 entries per M tile (its four accumulator rows)
    auto load_tg = [&](int64_t tile, uint2 (&dst)[MT]) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int mtile = mgrp * MT + mt;
            // an M tile past the last computes nothing (zero accumulators): the
            // targets of the last one are read and receive zeros
            const int mtc = mtile < mtiles ? mtile : mtiles - 1;
            dst[mt] = *reinterpret_cast<const uint2*>(tg16 + (((tile * mtiles + mtc) * 4 + ngrp) * 256 + lane * 4));
        }
    };

    // One tile: the loads of tile t + 1 (D rows into pf, targets into tn) are
    // issued first and stay in flight through the MFMAs and the integer adds of
    // tile t (targets tc, loaded one tile earlier); the loop is unrolled by two
    // so that the two target register sets alternate without copies. Past the
    // last tile the loads read the last tile again (unused).
    auto step = [&](int64_t t, const uint2 (&tc)[MT], uint2 (&tn)[MT]) {
        const bool more = t + 1 < ntiles;
        const int64_t tl = more ? t + 1 : t;
        issue(tl);
        load_tg(tl, tn);
        const __bf16* Dt = reinterpret_cast<const __bf16*>(dbase + (t & 1) * tsz);
        f4 acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[mt][v] = 0.f;
        const int c = ngrp * 16 + (lane & 15);
#pragma unroll
        for (int kb = 0; kb < KBMAX; ++kb) {
            if (kb < kb_count) {
                const bf8 b = *reinterpret_cast<const bf8*>(&Dt[TileLayout<MF>::at(kb * MF::K + (lane >> 4) * 8, c, Kp)]);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    if ((mgrp * MT + mt) < mtiles) acc[mt] = MF::mma(afr[mt][kb], b, acc[mt]);
            }
        }
        // fixed-point scatter: all conversions first, then the integer adds; the
        // entry's sign bit flips the float's sign bit before the rounding
        int q[MT][4];
        unsigned tgt[MT][4];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const unsigned w = v < 2 ? tc[mt].x : tc[mt].y;
                const unsigned e = (w >> (16 * (v & 1))) & 0xffffu;
                tgt[mt][v] = e & 0x7fffu;
                const float x = __uint_as_float(__float_as_uint(acc[mt][v]) ^ ((e & 0x8000u) << 16));
                q[mt][v] = __float2int_rn(x * scale);
            }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) atomicAdd(&sig[tgt[mt][v]], (unsigned)q[mt][v]);
        if (more) commit((int)((t + 1) & 1));
        __syncthreads();
    };
    uint2 tga[MT], tgb[MT];
    issue(0);
    load_tg(0, tga);
    commit(0);
    __syncthreads();
    for (int64_t t = 0; t < ntiles; t += 2) {
        step(t, tga, tgb);
        if (t + 1 < ntiles) step(t + 1, tgb, tga);
    }
    if (p.overwrite) {
        for (int64_t i = tid; i < p.Nb; i += nth) srow[i] = (TO)((double)(int)sig[i] * unit);
    } else {
        for (int64_t i = tid; i < p.Nb; i += nth) srow[i] = (TO)((double)srow[i] + (double)(int)sig[i] * unit);
    }
}

static int64_t abf_lds_bytes(int kb_count, int64_t Nb)
{
    const int Kp = kb_count * MfmaBF16::K;
    int64_t b = ((Nb + 64) * 4 + 15) / 16 * 16;
    b += 2 * (((int64_t)TileLayout<MfmaBF16>::size(Kp) * 2 + 15) / 16 * 16);
    b += (int64_t)Kp * 4 + 64;
    return b;
}

bool ab_bf16_fixed_fits(int64_t Nb, int sa, int Mp)
{
    const int kb_count = (sa + MfmaBF16::K - 1) / MfmaBF16::K;
    const int mtiles = Mp / 16;
    return Nb + 64 < 0x8000 && kb_count <= 4 && (mtiles + 2) / 3 <= 4 && kb_count * MfmaBF16::K * 8 <= 2 * 64 * ABF_WAVES &&
           abf_lds_bytes(kb_count, Nb) <= 160 * 1024 - 512 - 2 * ABF_WAVES * 8;
}

template <typename TO>
static hipError_t abf_launch(const AbParams& p, const void* Vt, const void* Cs, int64_t ldc, const double* rowmax,
                             const uint16_t* tg16, TO* sigma, hipStream_t st)
{
    if (p.Na <= 0 || p.Nb <= 0 || p.sa <= 0 || p.M <= 0) return hipSuccess;
    if (!rowmax || !tg16) return ab_invalid("alpha-beta: row maxima or 16-bit targets missing");
    if (!ab_bf16_fixed_fits(p.Nb, p.sa, p.Mp)) return ab_invalid("alpha-beta: shape outside the fixed-point BF16 kernel");
    const int kb_count = (p.sa + MfmaBF16::K - 1) / MfmaBF16::K;
    const int mtiles = p.Mp / 16;
    const int MT = (mtiles + 2) / 3;
    const size_t lds = (size_t)abf_lds_bytes(kb_count, p.Nb);
    const int64_t grid = (p.Na + 7) / 8 * 8;
#define ABF_GO(KBV, MTV)                                                                            \
    if (kb_count <= KBV && MT == MTV) {                                                             \
        auto kern = k_ab_bf16<TO, KBV, MTV>;                                                        \
        hipError_t e = hipFuncSetAttribute((const void*)kern,                                       \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
        if (e != hipSuccess) {                                                                      \
            set_launch_reason("hipFuncSetAttribute(max dynamic LDS) failed");                       \
            return e;                                                                               \
        }                                                                                           \
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * ABF_WAVES), lds, st, p,            \
                           (const __bf16*)Vt, (const __bf16*)Cs, ldc, rowmax, tg16, sigma, kb_count); \
        return hipGetLastError();                                                                   \
    }
    ABF_GO(1, 1)
    ABF_GO(2, 1)
    ABF_GO(3, 1)
    ABF_GO(4, 1)
    ABF_GO(1, 2)
    ABF_GO(2, 2)
    ABF_GO(3, 2)
    ABF_GO(4, 2)
    ABF_GO(1, 3)
    ABF_GO(2, 3)
    ABF_GO(3, 3)
    ABF_GO(4, 3)
    ABF_GO(1, 4)
    ABF_GO(2, 4)
    ABF_GO(3, 4)
    ABF_GO(4, 4)
#undef ABF_GO
    return ab_invalid("alpha-beta: no fixed-point BF16 kernel variant for this shape");
}

hipError_t launch_ab_bf16_fixed(const AbParams& p, const void* Vt, const void* Cs, int64_t ldc, const double* rowmax,
                                const uint16_t* tg16, double* sigma, hipStream_t st)
{
    return abf_launch<double>(p, Vt, Cs, ldc, rowmax, tg16, sigma, st);
}

hipError_t launch_ab_bf16_fixed(const AbParams& p, const void* Vt, const void* Cs, int64_t ldc, const double* rowmax,
                                const uint16_t* tg16, float* sigma, hipStream_t st)
{
    return abf_launch<float>(p, Vt, Cs, ldc, rowmax, tg16, sigma, st);
}

}  // namespace casci
