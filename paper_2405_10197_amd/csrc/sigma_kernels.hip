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
#include "ab_common.h"

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
template <>
struct Vec<float, 4> {
    using type = float4;
};

__device__ inline float bcast_val(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ inline double bcast_val(double v, int lane) { return bcast_f64(v, lane); }

#ifndef SS_GATHER_DEPTH
#define SS_GATHER_DEPTH 4
#endif
template <typename TX, typename TY, int LPE, int VW, typename TC, typename TV>
__global__ __launch_bounds__(256) void k_ss_gather(const TC* __restrict__ col,
                                                   const TV* __restrict__ val, int r,
                                                   int64_t nrows, int64_t ncols,
                                                   const TX* __restrict__ X, int64_t ldx,
                                                   TY* __restrict__ Y, double shift, int acc,
                                                   int64_t nrowblk, int64_t nitems, int64_t ipw)
{
    constexpr int G = 64 / LPE;
    static_assert(G == 1 || G == 2 || G == 4, "16, 32 or 64 lanes per entry");
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
        // this lane's VW consecutive columns (VW > 1 needs ldx % VW == 0: aligned
        // 8- or 16-byte loads)
        const int64_t c = (strip * LPE + li) * VW;
        const bool full = c + VW <= ncols;
        const bool cok = c < ncols;
        // one column per lane: lanes past the last column read column 0 (a valid
        // address) and discard the result, so the loads need no branch and the
        // compiler can keep D of them in flight
        const int64_t cl = cok ? c : 0;
        const TC* colI = col + I * (int64_t)r;
        const TV* valI = val + I * (int64_t)r;
        auto load = [&](int J, double* out) {
            const TX* src = X + (int64_t)J * ldx + c;
            if constexpr (VW == 1) {
                out[0] = (double)X[(int64_t)J * ldx + cl];
            } else {
                if (full) {
                    const VX v = *reinterpret_cast<const VX*>(src);
                    const TX* e = reinterpret_cast<const TX*>(&v);
#pragma unroll
                    for (int u = 0; u < VW; ++u) out[u] = (double)e[u];
                } else {
#pragma unroll
                    for (int u = 0; u < VW; ++u) out[u] = c + u < ncols ? (double)src[u] : 0.0;
                }
            }
        };
        // Summation order, the same for every strip width (so the result does
        // not depend on the autotuner's choice): accumulator a_k sums the
        // entries e = k mod 4 of the row in ascending order, and the row total is
        // (a_0 + a_1) + (a_2 + a_3). A lane of group g holds the accumulators of
        // its entries: all four (G = 1), k = g and g + 2 (G = 2), or k = g (G = 4).
        constexpr int NACC = VW == 1 ? SS_GATHER_DEPTH : 4;  // loads in flight per lane
        constexpr int NA = 4 / G;  // accumulators per lane
        double acc_[NA][VW] = {};
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
                if (VW == 1 || cok) {
                    double x[NACC][VW];
#pragma unroll
                    for (int h = 0; h < NACC; ++h) load(J[h], x[h]);
                    // entry j + h*G + g has e mod 4 = (h*G + g) mod 4: accumulator h mod NA
#pragma unroll
                    for (int h = 0; h < NACC; ++h)
#pragma unroll
                        for (int u = 0; u < VW; ++u) acc_[h % NA][u] += v[h] * x[h][u];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < VW; ++u) {
            double a;
            if constexpr (G == 1) {
                a = (acc_[0][u] + acc_[1][u]) + (acc_[NA - 2][u] + acc_[NA - 1][u]);
            } else if constexpr (G == 2) {
                const double lo = acc_[0][u] + __shfl_xor(acc_[0][u], LPE);       // a_0 + a_1
                const double hi = acc_[NA - 1][u] + __shfl_xor(acc_[NA - 1][u], LPE);  // a_2 + a_3
                a = lo + hi;
            } else {
                const double pr = acc_[0][u] + __shfl_xor(acc_[0][u], LPE);  // a_0 + a_1 | a_2 + a_3
                a = pr + __shfl_xor(pr, 2 * LPE);
            }
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

// ---------------------------------------------------------------------------
// row-blocked same-spin gather (strip width code SS_BLOCKED)
// ---------------------------------------------------------------------------
// One workgroup of SS_BLK_W = 16 waves takes 16 RW consecutive rows (RW = 1
// or 2 rows per wave) of a block of bk.rows = 16 or 32 and one strip of
// 64 x VW columns (VW adjacent columns per lane); wave w computes rows
// b*R + s*16*RW + w + 16q, q < RW, for part s of block b. The rows of X the block needs (the sorted union of its rows'
// columns) are staged into LDS, SS_BLK_CH at a time in two buffers (the loads
// of the next chunk are in flight while the current one is used), and each
// wave adds its rows' entry groups of the chunk, reading X from LDS.
// Neighbouring strings share most of their neighbours (at n = 16, 16 rows
// touch about 4000 distinct rows and 32 rows about 5400, against 849 entries
// per row), so each row of X crosses the L1 once per block instead of once per
// entry, and 32-row blocks stage a third fewer rows per row than 16-row ones.
//
// A group (four LDS byte offsets and four values) is wave-uniform scalar
// loads that feed the LDS reads and FMAs directly (the FP32-operator builds
// store (double)(float)v, the product the other widths form); the chunk
// offsets of a row sit in two registers (loaded once) and the union indices
// of a chunk are read ahead of its X rows, so the chunk loop waits on nothing
// it has just issued. Staged rows are SS_BLK_ROWB bytes apart whatever the
// element type and VW.
//
// The diagonal (entry 0, column I) comes from row I of X directly. Summation
// order: that of the other widths (accumulator k sums the entries e = k mod 4
// in ascending order, total (a0 + a1) + (a2 + a3)): the groups are aligned to
// the entry index, chunks ascend with the columns, and padded slots add v = 0;
// so the result does not depend on the block size either.
//
// TA is the accumulator type: double, or float for the BF16 build (groups
// with FP32 values, one FMA per entry and column without conversions; the
// same summation order in FP32).
#ifndef SS_BLK_WPE
#define SS_BLK_WPE 8
#endif
#ifndef SS_BLK_LDSB
#define SS_BLK_LDSB 1
#endif
template <typename TX, typename TY, typename TV, int VW, typename TA, int RW>
__global__ __launch_bounds__(64 * SS_BLK_W, SS_BLK_WPE) void k_ss_gather_blk(SsBlk bk,
                                                                 const SsGroupOf<TA>* __restrict__ gs,
                                                                 const TV* __restrict__ val, int r,
                                                                 int64_t nrows, int64_t ncols,
                                                                 const TX* __restrict__ X, int64_t ldx,
                                                                 TY* __restrict__ Y, double shift, int acc,
                                                                 int64_t nitems)
{
    constexpr int CH = SS_BLK_CH;
    constexpr int RPW = CH / SS_BLK_W;  // union rows a wave stages per chunk
    using VX = typename Vec<TX, VW>::type;
    using TG = SsGroupOf<TA>;
    constexpr int GB = RW == 2 && sizeof(TA) == 8 ? 2 : 4;  // groups per scalar round trip
    static_assert(64 * VW * sizeof(TX) <= SS_BLK_ROWB, "a staged row holds 64 x VW elements");
    extern __shared__ __align__(16) unsigned char smem[];  // [2][CH][SS_BLK_ROWB]
    const int64_t per_xcd = gridDim.x / 8;
    const int64_t t = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (t >= nitems) return;
    // item t: strip, block, and the part of the block this workgroup takes
    // (16 RW of its rows; a 32-row block is split in two when RW = 1)
    const int nsub = bk.rows / (SS_BLK_W * RW);
    const int64_t tb = t / nsub;
    const int sub = (int)(t - tb * nsub);
    const int64_t strip = tb / bk.nblk, b = tb - strip * bk.nblk;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t c = (strip * 64 + lane) * VW;
    const bool cok = c < ncols;
    // lanes past the last column read column 0 and store nothing; with VW = 2 the
    // row stride is even, so the pair (c, c + 1) lies inside the row
    const int64_t cl = cok ? c : 0;
    const int4 bi = bk.binfo[b];
    const uint16_t* U = bk.uni + bi.x;
    const int nU = bi.y, nch = bi.w;

    // per row of the wave: its index, the group offsets per chunk (lane l:
    // offset l and 64 + l) and the start of its group stream
    int64_t I[RW];
    bool rowok[RW];
    int o0[RW], o1[RW];
    const TG* grow[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        const int w = sub * SS_BLK_W * RW + wave + SS_BLK_W * q;  // row of the block
        I[q] = b * bk.rows + w;
        rowok[q] = I[q] < nrows;
        const uint16_t* goff = bk.goff + bi.z + (int64_t)w * (nch + 1);
        o0[q] = rowok[q] && lane <= nch ? (int)goff[lane] : 0;
        o1[q] = rowok[q] && 64 + lane <= nch ? (int)goff[64 + lane] : 0;
        grow[q] = gs + (rowok[q] ? (int64_t)bk.rbase[I[q]] : 0);
    }
    // both halves read and one selected: no branch per lookup
    auto off_at = [&](int q, int i) {
        const int lo = bcast_i32(o0[q], i & 63), hi = bcast_i32(o1[q], i & 63);
        return i < 64 ? lo : hi;
    };

    // Staging runs two chunks ahead: while chunk ch is used, the X rows of
    // chunk ch + 1 (registers of one set) and ch + 2 (the other set) are in
    // flight, and the union indices of chunk ch + 3 (lane i < RPW: the wave's
    // row i) are loaded before the X rows of ch + 2, so every wait leaves the
    // newer loads outstanding. The loop is unrolled by two so that the
    // register sets alternate statically.
    // The loads are unconditional and their results used as loaded, so that
    // the compiler's wait counts stay exact across the unrolled loop: slots
    // past the union stage row U[0] again, which no group refers to.
    auto load_u = [&](int ch) {
        const int k = ch * CH + wave * RPW + lane;
        return (int)U[k < nU ? k : 0];
    };
    // row offsets in 32 bits (the launch checks that every row of X is
    // within 2^32 elements), one scalar multiply per staged row
    const uint32_t ldx32 = (uint32_t)ldx;
    auto issue = [&](int un, VX (&pf)[RPW]) {
#pragma unroll
        for (int i = 0; i < RPW; ++i)
            pf[i] = *reinterpret_cast<const VX*>(X + (uint64_t)((uint32_t)bcast_i32(un, i) * ldx32) + cl);
    };
    auto commit = [&](int buf, const VX (&pf)[RPW]) {
#pragma unroll
        for (int i = 0; i < RPW; ++i)
            *reinterpret_cast<VX*>(smem + ((int64_t)buf * CH + wave * RPW + i) * SS_BLK_ROWB + lane * sizeof(VX)) =
                pf[i];
    };

    TA a[RW][VW][4] = {};
#pragma unroll
    for (int q = 0; q < RW; ++q)
#pragma unroll
        for (int u = 0; u < VW; ++u)
            if (rowok[q]) a[q][u][0] += (TA)val[I[q] * r] * (TA)X[I[q] * ldx + cl + u];
    auto compute = [&](int ch) {
        const unsigned char* sb = smem + (int64_t)(ch & 1) * CH * SS_BLK_ROWB + lane * sizeof(VX);
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            if (!rowok[q]) continue;
            auto add = [&](const TG& G) {
#if SS_BLK_LDSB >= 1
                VX xv[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) xv[k] = *reinterpret_cast<const VX*>(sb + G.off[k]);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const TX* xe = reinterpret_cast<const TX*>(&xv[k]);
#pragma unroll
                    for (int u = 0; u < VW; ++u) a[q][u][k] += G.v[k] * (TA)xe[u];
                }
#else
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const VX xv = *reinterpret_cast<const VX*>(sb + G.off[k]);
                    const TX* xe = reinterpret_cast<const TX*>(&xv);
#pragma unroll
                    for (int u = 0; u < VW; ++u) a[q][u][k] += G.v[k] * (TA)xe[u];
                }
#endif
            };
#if SS_BLK_LDSB == 4
            auto add4 = [&](const TG& G0, const TG& G1, const TG& G2, const TG& G3) {
                VX xv[4][4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    xv[0][k] = *reinterpret_cast<const VX*>(sb + G0.off[k]);
                    xv[1][k] = *reinterpret_cast<const VX*>(sb + G1.off[k]);
                    xv[2][k] = *reinterpret_cast<const VX*>(sb + G2.off[k]);
                    xv[3][k] = *reinterpret_cast<const VX*>(sb + G3.off[k]);
                }
                const TG* GG[4] = {&G0, &G1, &G2, &G3};
#pragma unroll
                for (int h = 0; h < 4; ++h)
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const TX* xe = reinterpret_cast<const TX*>(&xv[h][k]);
#pragma unroll
                        for (int u = 0; u < VW; ++u) a[q][u][k] += GG[h]->v[k] * (TA)xe[u];
                    }
            };
#endif
            const TG* gr = grow[q];
            const int g1 = off_at(q, ch + 1);
            int g = off_at(q, ch);
            // up to four groups per scalar round trip (two with two FP64 rows
            // per wave, whose scalar registers would spill otherwise)
            if constexpr (GB == 4) {
                for (; g + 4 <= g1; g += 4) {
                    const TG G0 = gr[g], G1 = gr[g + 1], G2 = gr[g + 2], G3 = gr[g + 3];
#if SS_BLK_LDSB == 4
                    add4(G0, G1, G2, G3);
#else
                    add(G0);
                    add(G1);
                    add(G2);
                    add(G3);
#endif
                }
            }
            for (; g + 2 <= g1; g += 2) {
                const TG G0 = gr[g], G1 = gr[g + 1];
                add(G0);
                add(G1);
            }
            if (g < g1) add(gr[g]);
        }
    };
    // one chunk: pn holds the X rows of chunk ch + 1 (in flight), pf receives
    // those of chunk ch + 2 from the indices un; the indices of ch + 3 go to un2
    // L2 prefetch of the next chunk's group data: one coalesced dword per lane
    // and row (256 bytes) whose value is folded into a dummy one step later
    // (and the dummy kept alive by an empty asm statement at the end), so the
    // scalar loads of that chunk find their lines in the L2 instead of the
    // memory side: 44.6 -> 40.6 ms (FP64) and 24.7 -> 23.1 ms (FP32 input,
    // FP64 sums) at CAS(16,16) with 16-row blocks; two chunks ahead was slower
    const int gw = (int)(sizeof(TG) / 4);  // dwords per group
    // last dword of each row's groups (rows past the last have none: index 0
    // of the stream, which exists)
    int gend[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) gend[q] = max(off_at(q, nch) * gw - 1, 0);
    unsigned pfx[RW], pfx_acc = 0u;
#pragma unroll
    for (int q = 0; q < RW; ++q) pfx[q] = 0u;
    auto step = [&](int ch, VX (&pn)[RPW], VX (&pf)[RPW], int& un, int& un2) {
        un2 = load_u(ch + 3);
        issue(un, pf);
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            pfx_acc ^= pfx[q];
            const int i = off_at(q, ch + 1 < nch ? ch + 1 : ch) * gw + lane;
            pfx[q] = reinterpret_cast<const unsigned*>(grow[q])[i < gend[q] ? i : gend[q]];
        }
        compute(ch);
        if (ch + 1 < nch) commit((ch + 1) & 1, pn);
        __syncthreads();
    };
    VX pa[RPW], pb[RPW];
    int ua = load_u(0);
    int ub = load_u(1);
    issue(ua, pa);
    issue(ub, pb);
    ua = load_u(2);
    commit(0, pa);
    __syncthreads();
    // chunk ch (even): next rows in pb, rows of ch + 2 into pa from ua, indices of ch + 3 into ub
    for (int ch = 0; ch < nch; ch += 2) {
        step(ch, pb, pa, ua, ub);
        if (ch + 1 < nch) step(ch + 1, pa, pb, ub, ua);
    }
#pragma unroll
    for (int q = 0; q < RW; ++q) pfx_acc ^= pfx[q];
    asm volatile("" ::"v"(pfx_acc));
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        if (!rowok[q]) continue;
#pragma unroll
        for (int u = 0; u < VW; ++u) {
            if (c + u >= ncols) continue;
            const int64_t o = I[q] * ncols + c + u;
            // the diagonal element again (not held in registers through the loop)
            const double xI = (double)X[I[q] * ldx + cl + u];
            double y = (double)((a[q][u][0] + a[q][u][1]) + (a[q][u][2] + a[q][u][3])) + shift * xI;
            if (acc) y += (double)Y[o];
            Y[o] = (TY)y;
        }
    }
}

template <typename TX, typename TY, typename TV, typename TA = double>
static hipError_t ss_gather_blk(const SsBlk& bk, const SsGroupOf<TA>* gs, const TV* val, int r, int64_t nrows,
                                int64_t ncols, const TX* X, int64_t ldx, TY* Y, double shift, int acc, hipStream_t st)
{
    if (nrows <= 0 || ncols <= 0) return hipSuccess;
    if (!bk.uni || !gs || bk.ch != SS_BLK_CH) return invalid("same-spin gather: no row-blocked operator");
    if (bk.rows != SS_BLK_W && bk.rows != 2 * SS_BLK_W) return invalid("same-spin gather: unsupported block size");
    // a prefix of the rows (the autotuner times one) takes the blocks that cover it
    SsBlk b = bk;
    b.nblk = (nrows + bk.rows - 1) / bk.rows;
    if (b.nblk > bk.nblk) return invalid("same-spin gather: more rows than the row-blocked operator has");
    // staged rows are addressed with 32-bit element offsets
    if ((uint64_t)bk.nblk * (uint64_t)bk.rows * (uint64_t)ldx >= ((uint64_t)1 << 32))
        return invalid("same-spin gather: X too large for the row-blocked form's 32-bit row offsets");
    // FP32 input: two adjacent columns per lane when the row stride allows aligned pairs
    const bool pair = sizeof(TX) == 4 && ldx % 2 == 0;
    const int64_t nstrip = (ncols + (pair ? 127 : 63)) / (pair ? 128 : 64);
    // two rows per wave on 32-row blocks, except where the FP64 sums of
    // column pairs would not fit the registers of 8 waves per SIMD (then two
    // workgroups share a block, each staging its union)
    const bool two = bk.rows == 2 * SS_BLK_W && !(pair && sizeof(TA) == 8);
    const int nsub = bk.rows / (SS_BLK_W * (two ? 2 : 1));
    const int64_t nitems = nstrip * b.nblk * nsub;
    if (nitems > ((int64_t)1 << 31) - 8) return invalid("same-spin gather: too many row blocks x strips");
    const int64_t grid = (nitems + 7) / 8 * 8;
    const size_t lds = (size_t)2 * SS_BLK_CH * SS_BLK_ROWB;
    auto launch = [&](auto kern) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return invalid("hipFuncSetAttribute(max dynamic LDS) failed");
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * SS_BLK_W), lds, st, b, gs, val, r, nrows, ncols, X,
                           ldx, Y, shift, acc, nitems);
        return hipGetLastError();
    };
    if constexpr (sizeof(TX) == 4) {
        if (pair) {
            if constexpr (sizeof(TA) == 8)
                return launch(k_ss_gather_blk<TX, TY, TV, 2, TA, 1>);
            else
                return two ? launch(k_ss_gather_blk<TX, TY, TV, 2, TA, 2>)
                           : launch(k_ss_gather_blk<TX, TY, TV, 2, TA, 1>);
        }
    }
    return two ? launch(k_ss_gather_blk<TX, TY, TV, 1, TA, 2>) : launch(k_ss_gather_blk<TX, TY, TV, 1, TA, 1>);
}

// strip width code: 16 / 32 / 64 lanes per entry with one column each, 128 =
// 64 lanes with two adjacent columns each, or LPE * 100 + VW for LPE lanes per
// entry with VW adjacent columns each (1602, 3202: 16-byte loads of FP64 pairs
// with 4 or 2 entries per wave-wide load; 1604, 3204, 6404: FP32 quadruples).
// A vector width the row stride does not allow falls back to one column per
// lane. The summation order is the same for every code.
template <typename TX, typename TY, typename TC, typename TV>
static hipError_t ss_gather_w(const TC* col, const TV* val, int r, int64_t nrows, int64_t ncols,
                              const TX* X, int64_t ldx, TY* Y, double shift, int acc, hipStream_t st, int lpe)
{
    constexpr bool f32 = sizeof(TX) == 4;
    switch (lpe) {
    case 16: return ss_gather<TX, TY, 16, 1>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
    case 32: return ss_gather<TX, TY, 32, 1>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
    case 0:
    case 64: return ss_gather<TX, TY, 64, 1>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
    case 128:
        if (ldx % 2 != 0) return ss_gather<TX, TY, 64, 1>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
        return ss_gather<TX, TY, 64, 2>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
    case 1602:
        if (ldx % 2 != 0) return ss_gather<TX, TY, 16, 1>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
        return ss_gather<TX, TY, 16, 2>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
    case 3202:
        if (ldx % 2 != 0) return ss_gather<TX, TY, 32, 1>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
        return ss_gather<TX, TY, 32, 2>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
    case 1604:
    case 3204:
    case 6404:
        if constexpr (f32) {
            if (ldx % 4 == 0) {
                if (lpe == 1604) return ss_gather<TX, TY, 16, 4>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
                if (lpe == 3204) return ss_gather<TX, TY, 32, 4>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
                return ss_gather<TX, TY, 64, 4>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
            }
        }
        return ss_gather<TX, TY, 64, 1>(col, val, r, nrows, ncols, X, ldx, Y, shift, acc, st);
    default: return invalid("same-spin gather: unknown strip width code");
    }
}

hipError_t launch_ss_gather_f64(const SsOp& op, int64_t nrows, int64_t ncols, const double* X, double* Y,
                                double shift, int acc, hipStream_t st, int lpe)
{
    if (lpe == SS_BLOCKED && op.blk.uni)
        return ss_gather_blk<double, double>(op.blk, op.blk.gs64, op.val, op.r, nrows, ncols, X, ncols, Y, shift,
                                             acc, st);
    if (lpe == SS_BLOCKED) lpe = 64;
    if (op.col16)
        return ss_gather_w<double, double>(op.col16, op.val, op.r, nrows, ncols, X, ncols, Y, shift, acc, st, lpe);
    return ss_gather_w<double, double>(op.col, op.val, op.r, nrows, ncols, X, ncols, Y, shift, acc, st, lpe);
}

hipError_t launch_ss_gather_f32in(const SsOp& op, int64_t nrows, int64_t ncols, const float* X, int64_t ldx,
                                  double* Y, double shift, int acc, hipStream_t st, int lpe, bool acc32)
{
    if (lpe == SS_BLOCKED && op.blk.uni && op.val32 && acc32 && op.blk.gsf)
        return ss_gather_blk<float, double, float, float>(op.blk, op.blk.gsf, op.val32, op.r, nrows, ncols, X, ldx, Y,
                                                          shift, acc, st);
    if (lpe == SS_BLOCKED && op.blk.uni && op.val32)
        return ss_gather_blk<float, double>(op.blk, op.blk.gs32, op.val32, op.r, nrows, ncols, X, ldx, Y, shift,
                                            acc, st);
    if (lpe == SS_BLOCKED) lpe = 64;
    if (op.col16 && op.val32)
        return ss_gather_w<float, double>(op.col16, op.val32, op.r, nrows, ncols, X, ldx, Y, shift, acc, st, lpe);
    return ss_gather_w<float, double>(op.col, op.val, op.r, nrows, ncols, X, ldx, Y, shift, acc, st, lpe);
}

hipError_t launch_ss_gather_f32(const SsOp& op, int64_t nrows, int64_t ncols, const float* X, float* Y,
                                double shift, int acc, hipStream_t st, int lpe)
{
    if (lpe == SS_BLOCKED && op.blk.uni && op.val32)
        return ss_gather_blk<float, float>(op.blk, op.blk.gs32, op.val32, op.r, nrows, ncols, X, ncols, Y, shift,
                                           acc, st);
    if (lpe == SS_BLOCKED) lpe = 64;
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
// nrm2 (may be null): nrm2[block] = sum of the squares of the values the
// block wrote (fixed order), for a norm of the result without another pass
__global__ __launch_bounds__(256) void k_sym_add(double* __restrict__ S, int64_t n, double p,
                                                 double scale, int64_t nb, const double* __restrict__ T,
                                                 double* __restrict__ nrm2)
{
    __shared__ double A[32][33];
    __shared__ double B[32][33];
    int64_t bi, bj;
    tile_pair_of(blockIdx.x, nb, bi, bj);
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t r0 = bi * 32, c0 = bj * 32;
    for (int i = ty; i < 32; i += 8) {
        const int64_t ra = r0 + i, ca = c0 + tx;
        A[i][tx] = (ra < n && ca < n) ? S[ra * n + ca] : 0.0;
        const int64_t rb = c0 + i, cb = r0 + tx;
        B[i][tx] = (rb < n && cb < n) ? S[rb * n + cb] : 0.0;
    }
    __syncthreads();
    double ss = 0.0;
    for (int i = ty; i < 32; i += 8) {
        const int64_t ra = r0 + i, ca = c0 + tx;
        if (ra < n && ca < n) {
            const double y = scale * (A[i][tx] + p * B[tx][i]) + (T ? T[ra * n + ca] : 0.0);
            S[ra * n + ca] = y;
            ss += y * y;
        }
        if (bi != bj) {
            const int64_t rb = c0 + i, cb = r0 + tx;
            if (rb < n && cb < n) {
                const double y = scale * (B[i][tx] + p * A[tx][i]) + (T ? T[rb * n + cb] : 0.0);
                S[rb * n + cb] = y;
                ss += y * y;
            }
        }
    }
    if (nrm2) {  // uniform: the whole block takes this branch or none
        __syncthreads();
        double* red = &A[0][0];
        red[threadIdx.x] = ss;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) nrm2[blockIdx.x] = red[0];
    }
}

hipError_t launch_sym_add(double* S, int64_t n, int p, double scale, hipStream_t st, const double* T,
                          double* nrm2)
{
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 31) / 32;
    const int64_t pairs = nb * (nb + 1) / 2;
    if (pairs > 0x7fffffffLL) return invalid("sym_add: matrix too large");
    hipLaunchKernelGGL(k_sym_add, dim3((unsigned)pairs), dim3(256), 0, st, S, n, (double)p, scale, nb, T, nrm2);
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
// alpha-beta scatter targets (shared by the FP64 and low-precision kernels)
// ---------------------------------------------------------------------------
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

// C (FP64 or FP32, rows x cols) -> padded copy in the MFMA input type, row stride ld
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

int abl_waves(int Mp)
{
    (void)Mp;
    return ABL_MAX_WAVES;  // 4 column groups x 3 pair-row groups
}

hipError_t launch_ab_lowp(const AbParams& p, const AbReduce& r, int prec, const void* Vt, const void* Cs,
                          int64_t ldc, double* sigma, hipStream_t st)
{
    if (prec == 1) return launch_ab_lowp_f32(p, r, Vt, Cs, ldc, sigma, st);
    if (prec == 2) return launch_ab_lowp_bf16(p, r, Vt, Cs, ldc, sigma, st);
    return invalid("alpha-beta: unknown precision");
}

hipError_t launch_ab_lowp(const AbParams& p, const AbReduce& r, int prec, const void* Vt, const void* Cs,
                          int64_t ldc, float* sigma, hipStream_t st)
{
    if (prec == 1) return launch_ab_lowp_f32(p, r, Vt, Cs, ldc, sigma, st);
    if (prec == 2) return launch_ab_lowp_bf16(p, r, Vt, Cs, ldc, sigma, st);
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
