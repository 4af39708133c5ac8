#include "common.h"
extern "C" {
size_t sl_mlp_workspace_size(int batch) { return 0; }
int sl_mlp_forward(const float*, const float*, int, float*, void*, void*) { return SL_ENOIMPL; }
int sl_mlp_train_step(float*, float*, float*, const float*, const float*, int, float, int, float*, float*,
                      void*, void*) { return SL_ENOIMPL; }
}
