// Trace-kernel instances for rocking curves whose shift and width depend on
// the photon energy (sec. 2.2.1): both precisions, records on and off, every
// geometry and kind read at run time.
#include "trace_impl.h"

namespace mrt {

const void *edep_kernel_ptr(int precision, bool records) {
    if (precision == MRT_FP64)
        return records ? (const void *)tk::trace_kernel_edep<double, true>
                       : (const void *)tk::trace_kernel_edep<double, false>;
    return records ? (const void *)tk::trace_kernel_edep<float, true>
                   : (const void *)tk::trace_kernel_edep<float, false>;
}

}  // namespace mrt
