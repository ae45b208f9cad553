// Trace-kernel instances for the extended inputs (an energy-dependent rocking
// curve, sec. 2.2.1; a finite source spot and user ray arrays, sec. 2.1):
// both precisions, records on and off, every geometry and kind read at run
// time.
#include "trace_impl.h"

namespace mrt {

const void *ext_kernel_ptr(int precision, bool records) {
    if (precision == MRT_FP64)
        return records ? (const void *)tk::trace_kernel_ext<double, true>
                       : (const void *)tk::trace_kernel_ext<double, false>;
    return records ? (const void *)tk::trace_kernel_ext<float, true>
                   : (const void *)tk::trace_kernel_ext<float, false>;
}

}  // namespace mrt
