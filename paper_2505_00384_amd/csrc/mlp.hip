// Learned per-cell preconditioner (network kernels).
#include "common.hpp"

namespace hx {

struct MlpState {
    int dummy;
};

hx_status mlp_create(hx_ctx *c) { return fail(c, HX_ERR_STATE, "network not available"); }
void mlp_destroy(hx_ctx *c) { (void)c; }
int64_t mlp_param_count(const hx_ctx *c)
{
    const int64_t ni = c->nd + 6 * c->nf + 1, h = 256, no = c->nd;
    return h * ni + h + h * h + h + no * h + no;
}
hx_status mlp_set(hx_ctx *c, const float *, int64_t) { return fail(c, HX_ERR_STATE, "network not available"); }
hx_status mlp_get(const hx_ctx *c, float *, int64_t) { (void)c; return HX_ERR_STATE; }
hx_status mlp_features(hx_ctx *c, const double *, float *, float *) { return fail(c, HX_ERR_STATE, "network not available"); }
hx_status mlp_forward(hx_ctx *c, const float *, int64_t, float *) { return fail(c, HX_ERR_STATE, "network not available"); }
hx_status mlp_train(hx_ctx *c, const float *, const float *, int64_t, float, float *, float *)
{
    return fail(c, HX_ERR_STATE, "network not available");
}
hx_status mlp_precondition(hx_ctx *c, const double *, double *, int *)
{
    return fail(c, HX_ERR_STATE, "network not available");
}

}  // namespace hx
