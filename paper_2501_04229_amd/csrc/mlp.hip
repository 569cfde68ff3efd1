// (alpha, omega) predictor: placeholder entry points until the MLP kernels land.
#include "internal.h"

extern "C" {
gadi_status gadi_mlp_create(uint64_t, gadi_mlp** out) { if (out) *out = nullptr; return GADI_EINVAL; }
gadi_status gadi_mlp_destroy(gadi_mlp*) { return GADI_EINVAL; }
gadi_status gadi_mlp_set_weights(gadi_mlp*, const float*) { return GADI_EINVAL; }
gadi_status gadi_mlp_get_weights(gadi_mlp*, float*) { return GADI_EINVAL; }
gadi_status gadi_mlp_set_norm(gadi_mlp*, const float*, const float*) { return GADI_EINVAL; }
gadi_status gadi_mlp_forward(gadi_mlp*, const float*, int32_t, float*) { return GADI_EINVAL; }
gadi_status gadi_mlp_loss_grad(gadi_mlp*, const float*, const float*, int32_t, float*, float*) { return GADI_EINVAL; }
gadi_status gadi_train_mlp(gadi_mlp*, const float*, const float*, int32_t, int32_t, float, float*) { return GADI_EINVAL; }
gadi_status gadi_predict_params(gadi_mlp*, const float*, double*, double*) { return GADI_EINVAL; }
}
