// Trace-kernel instances: double precision, flat crystal, every mosaic
// distribution x rocking curve x records combination.
#include "trace_impl.h"

namespace mrt {
MRT_TRACE_TABLE(trace_table_f64_flat, double, MRT_GEOMETRY_FLAT)
}  // namespace mrt
