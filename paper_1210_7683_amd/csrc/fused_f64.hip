// Instantiations of the fused contraction + solve kernel for one form, p = 2..20.
#include "fused_dma.h"

namespace gw {

hipError_t launch_fused_f64(const FusedArgs &a, hipStream_t s) {
    return dispatch_dma<GWAS_FORM_F64, false>(a, s);
}

}  // namespace gw
