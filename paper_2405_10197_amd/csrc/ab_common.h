// Device code shared by the alpha-beta contraction kernels (FP64 in
// ab_f64.hip, FP32/BF16 in ab_lowp_*.hip): MFMA operand types, the layout of
// the LDS tile of gathered C rows, and launch helpers.
//
// The contraction (row-blocked form of the alpha-beta term of the sigma build,
// Sec. II.A.1): for one alpha string Ia and a tile of TN beta strings Jb,
//   D(e, Jb) = C(J_e, Jb)                 e in L1(Ia)  (row gathers -> LDS)
//   T(m, Jb) = sum_e A(m, e) D(e, Jb)     A(m, e) = s_e (p_e q_e | r_m s_m)
//   sigma(Ia, Ib) += sign T(m, Jb)        Ib = E_{r_m s_m} Jb
// Pair rows m: r <= s when the integrals are symmetric in rs (T(rs) = T(sr);
// the one of E_rs / E_sr that does not vanish on Jb is applied), or all
// ordered (r, s) when an S^2 penalty (not rs-symmetric) is folded in.
#pragma once

#include "internal.h"

#include <climits>

namespace casci {

inline hipError_t ab_invalid(const char* why)
{
    set_launch_reason(why);
    return hipErrorInvalidValue;
}

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

constexpr int AB_MAX_WAVES = 12;   // FP64 kernel: one 16-row M tile per wave (two above 12 tiles)
constexpr int ABL_MAX_WAVES = 12;  // low-precision kernel: 4 column groups x 3 pair-row groups

}  // namespace casci
