// Trace-kernel instances: double precision, cylindrical crystal, every mosaic
// distribution x rocking curve x records combination.
#include "trace_impl.h"

namespace mrt {
MRT_TRACE_TABLE(trace_table_f64_cyl, double, MRT_GEOMETRY_CYLINDER)
}  // namespace mrt
