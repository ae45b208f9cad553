// Serving-kernel instances, double precision: the plain one (each item in the
// loop specialised for its kinds) and the extended one.
#include "serve_kernels.h"

namespace mrt {

const void *serve_kernel_ptr_f64(bool ext) {
    return ext ? (const void *)tk::serve_kernel_ext<double> : (const void *)tk::serve_kernel<double>;
}

}  // namespace mrt
