// Low-precision alpha-beta contraction kernel (FP32 or BF16 MFMA, FP32
// accumulation) and its launcher, instantiated once per MFMA type in
// ab_lowp_f32.hip and ab_lowp_bf16.hip.
#pragma once

#include "ab_common.h"

namespace casci {

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

// layout of the low-precision kernel's waves: NS 16-column sub-tiles per wave
// (1: 4 column groups x 3 row groups; 4: one column group x 12 row groups)
// and MT 16-row M tiles per wave
// afr_regs: registers of one M tile's A fragments (kb_count operands). The
// column-group layout gives a wave up to four M tiles; when their fragments
// would take more than 64 registers (FP32 at n = 18: 4 x 23) the kernel
// spills, and the one-tile-per-wave layout is used instead.
inline void abl_layout(int Mp, int afr_regs, int& NS, int& MT)
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
inline int64_t abl_lds_bytes(int kb_count, int ldT, int max_nseg, int64_t chunk)
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
inline hipError_t abl_launch(const AbParams& p, const AbReduce& r, const void* Vt, const void* Cs, int64_t ldc,
                             TO* sigma, hipStream_t st)
{
    if (p.Na <= 0 || p.Nb <= 0 || p.sa <= 0 || p.M <= 0) return hipSuccess;
    if (r.ldT < p.Mp + 4 || (int64_t)AB_TN * r.ldT + 1 > 0x7fff || r.ldT % 4 != 0)
        return ab_invalid("alpha-beta: T tile stride does not fit the table's 15-bit offsets");
    if (p.Nb >= 0xffff) return ab_invalid("alpha-beta: more than 65534 beta strings for the low-precision table");
    const int kb_count = (p.sa + MF::K - 1) / MF::K;
    const int nwaves = abl_waves(p.Mp);
    int NS = 1, MT = 1;
    abl_layout(p.Mp, kb_count * (int)(sizeof(typename MF::frag) / 4), NS, MT);
    if (NS == 4 && MT > 2) return ab_invalid("alpha-beta: too many pair rows (norb too large)");
    const int64_t fixed = abl_lds_bytes<MF>(kb_count, r.ldT, r.max_nseg, 0);
    const int64_t cap = 160 * 1024 - 512;
    int64_t chunk = (cap - fixed) / 4;
    if (chunk < 256) return ab_invalid("alpha-beta: LDS too small for the sigma row chunk");
    int nchunks = (int)((p.Nb + chunk - 1) / chunk);
    chunk = (p.Nb + nchunks - 1) / nchunks;
    const size_t lds = (size_t)abl_lds_bytes<MF>(kb_count, r.ldT, r.max_nseg, chunk);
    const int nseg = kb_count * MF::K * (AB_TN * (int)sizeof(typename MF::elem) / 16) + r.max_nseg;
    const int spt = (nseg + 64 * nwaves - 1) / (64 * nwaves);
    if (spt > 8) return ab_invalid("alpha-beta: tile larger than the prefetch registers");
    const int64_t items = p.Na * nchunks;
    const int64_t grid = (items + 7) / 8 * 8;
    dim3 blk(64 * nwaves);
#define ABL_GO(KBV, MTV, SPTV, NSV)                                                                 \
    {                                                                                               \
        auto kern = k_ab_lp<MF, KBV, MTV, SPTV, TO, NSV>;                                           \
        hipError_t e = hipFuncSetAttribute((const void*)kern,                                       \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
        if (e != hipSuccess) {                                                                      \
            set_launch_reason("hipFuncSetAttribute(max dynamic LDS) failed");                       \
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
    return ab_invalid("alpha-beta: no kernel variant for this K-block count");
}

// C (FP64, rows x cols) -> padded copy in the MFMA input type, row stride ld

}  // namespace casci
