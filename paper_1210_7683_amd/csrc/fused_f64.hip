// Instantiations of the fused contraction + solve kernel for one form, p = 2..20.
#include "fused.h"

namespace gw {

hipError_t launch_fused_f64(const FusedArgs &a, hipStream_t s) {
    return dispatch_p<GWAS_FORM_F64, false>(a, s);
}

}  // namespace gw
