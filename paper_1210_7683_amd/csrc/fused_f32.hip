// Instantiations of the fused contraction + solve kernel for one form, p = 2..20.
#include "fused.h"

namespace gw {

hipError_t launch_fused_f32(const FusedArgs &a, hipStream_t s) {
    if (a.f32_flush > 0) return dispatch_p<GWAS_FORM_F32, true>(a, s);
    return dispatch_p<GWAS_FORM_F32, false>(a, s);
}

}  // namespace gw
