// Matrix-core product kernels for X stored as __hip_bfloat16.
#include "prod_mfma.h"

namespace nmf {
namespace mfma {

void launch_bf16(int rp, int L, const ProdArgs &a, hipStream_t s)
{
#define NMF_L(RPV)                                               \
    if (L == 2) launch_mfma<RPV, __hip_bfloat16, 2>(a, s);                 \
    else launch_mfma<RPV, __hip_bfloat16, 1>(a, s);
    switch (rp) {
    case 16: NMF_L(16) break;
    case 32: NMF_L(32) break;
    case 48: NMF_L(48) break;
    case 64: NMF_L(64) break;
    default: break;
    }
#undef NMF_L
}

}  // namespace mfma
}  // namespace nmf
