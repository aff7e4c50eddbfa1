// Post-training quantisation of a loaded material (Sec. 5.2, "Precision").
#include <hip/hip_runtime.h>

#include <cstring>

#include "nam_internal.h"

using namespace nam;

extern "C" nam_status nam_material_set_precision(nam_ctx* ctx, nam_material* m, nam_dtype weights, nam_dtype texels,
                                                 const float* act_absmax, int first_layer_f16) {
    (void)act_absmax;
    (void)first_layer_f16;
    if (!ctx || !m) return set_error(NAM_E_INVALID_ARG, "NULL handle");
    if (weights == NAM_F32) {
        if (texels != NAM_F32) return set_error(NAM_E_UNSUPPORTED, "FP32 weights need FP32 texels");
        m->wprec = NAM_F32;
        m->tprec = NAM_F32;
        return NAM_OK;
    }
    return set_error(NAM_E_UNSUPPORTED, "low-precision decode is not available in this build");
}
