// Instantiations of the fused contraction + solve kernels for one form, p = 2..20.
#include "fused_dma.h"
#include "fused_wide.h"

namespace gw {

hipError_t launch_fused_bf16(const FusedArgs &a, hipStream_t s) {
    switch (a.p) {   // the wide-block tile where its accumulators fit the registers
    case 2: return launch_bf16_wide<2>(a, s);
    case 3: return launch_bf16_wide<3>(a, s);
    case 4: return launch_bf16_wide<4>(a, s);
    default: return dispatch_dma<GWAS_FORM_BF16X3, false>(a, s);
    }
}

}  // namespace gw
