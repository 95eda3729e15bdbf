// Instantiations of the fused contraction + solve kernels for one form, p = 2..20.
#include "fused_dma.h"

namespace gw {

hipError_t launch_fused_bf16x6(const FusedArgs &a, hipStream_t s) {
    return dispatch_dma<GWAS_FORM_BF16X6, true>(a, s);
}

}  // namespace gw
