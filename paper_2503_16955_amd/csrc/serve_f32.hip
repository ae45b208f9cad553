// Serving-kernel instances, FP32-mixed precision: the plain one (each item in the
// loop specialised for its kinds) and the extended one.
#include "serve_kernels.h"

namespace mrt {

const void *serve_kernel_ptr_f32(bool ext) {
    return ext ? (const void *)tk::serve_kernel_ext<float> : (const void *)tk::serve_kernel<float>;
}

}  // namespace mrt
