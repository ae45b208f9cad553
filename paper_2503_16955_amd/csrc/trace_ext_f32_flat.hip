// Extended-input trace-kernel instances (energy-dependent rocking curve,
// sec. 2.2.1; polarisations, sec. 2.1 and 2.2.3-2.2.4; further plane sets,
// sec. 2.2.3): FP32-mixed precision, flat crystal, every mosaic distribution x rocking
// curve x records combination.
#include "trace_impl.h"

namespace mrt {
MRT_EXT_TABLE(ext_table_f32_flat, float, MRT_GEOMETRY_FLAT)
}  // namespace mrt
