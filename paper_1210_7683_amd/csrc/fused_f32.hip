// Instantiations of the fused contraction + solve kernels for one form, p = 2..20.
#include "fused_dma.h"
#include "fused_gemv.h"

namespace gw {

hipError_t launch_fused_f32(const FusedArgs &a, hipStream_t s) {
    if (a.small_t) return dispatch_gemv<GWAS_FORM_F32>(a, s);
    if (a.f32_flush > 0) return dispatch_dma<GWAS_FORM_F32, true>(a, s);
    return dispatch_dma<GWAS_FORM_F32, false>(a, s);
}

}  // namespace gw
