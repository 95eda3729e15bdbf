// Instantiations of the fused contraction + solve kernel for one form, p = 2..20.
#include "fused.h"

namespace gw {

hipError_t launch_fused_bf16(const FusedArgs &a, hipStream_t s) {
    return dispatch_p<GWAS_FORM_BF16X3, false>(a, s);
}

}  // namespace gw
