// BF16 alpha-beta contraction into an FP32 sigma (FP32-storage builds): one instance of the
// low-precision kernel of ab_lowp.h (one file per instance so that they
// compile in parallel).
#include "ab_lowp.h"

namespace casci {

hipError_t launch_ab_lowp_bf16(const AbParams& p, const AbReduce& r, const void* Vt, const void* Cs, int64_t ldc,
                            float* sigma, hipStream_t st)
{
    return abl_launch<MfmaBF16, float>(p, r, Vt, Cs, ldc, sigma, st);
}

}  // namespace casci
