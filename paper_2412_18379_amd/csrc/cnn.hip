#include "common.h"

namespace cnnsns {

void run_predict(const cnnsns_mesh_s&, const float*, const cnnsns_cnn&, int32_t, float*, hipStream_t)
{
    fail(CNNSNS_EINVAL, "predict: CNN kernels not available in this build");
}

}  // namespace cnnsns
