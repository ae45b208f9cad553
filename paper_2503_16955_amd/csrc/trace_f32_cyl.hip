// Trace-kernel instances: float precision, cylindrical crystal, every mosaic
// distribution x rocking curve x records combination.
#include "trace_impl.h"

namespace mrt {
MRT_TRACE_TABLE(trace_table_f32_cyl, float, MRT_GEOMETRY_CYLINDER)
}  // namespace mrt
