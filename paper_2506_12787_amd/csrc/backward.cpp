// Backward pass entry point (blend -> preprocess -> MLP).
#include "runtime.h"

using namespace swf;

extern "C" swf_status swf_render_backward(swf_ctx* h, int32_t scene_id, const float* tx, int32_t batch, int32_t flags,
                                          const float* grad_out, const void* aux, const swf_grads* grads,
                                          void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return SWF_E_INVALID;
    (void)scene_id; (void)tx; (void)batch; (void)flags; (void)grad_out; (void)aux; (void)grads; (void)stream;
    return c->fail(SWF_E_STATE, "backward pass is not available in this build");
}
