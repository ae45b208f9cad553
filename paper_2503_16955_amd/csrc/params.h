// Validation of the public structs and the kernels' parameter block
// (shared by the one-call path and the request server).
#pragma once
#include <vector>

#include "mosaicrt.h"
#include "trace_params.h"

namespace mrt {

// Error reporter: records a formatted message and returns the status.
typedef mrt_status (*Failer)(mrt_status, const char *, ...);

// The library's reporter: the message becomes this thread's mrt_last_error().
mrt_status fail(mrt_status s, const char *fmt, ...);
const char *last_error();
void clear_error();

// EINVAL with a message (through `fail`) for an invalid combination.
mrt_status validate(const mrt_source *s, const mrt_crystal *c, const mrt_mosaic *m,
                    const mrt_rocking_curve *r, const mrt_detector *d, Failer fail);

// Fill the parameter block (geometry in crystal-local coordinates); `tables`
// receives the rocking-curve table followed by the spectrum CDF.  The run
// fields (ray range, seed, buffers, counters) are left to the caller.
void build_params(const mrt_source *s, const mrt_crystal *c, const mrt_mosaic *m,
                  const mrt_rocking_curve *r, const mrt_detector *d, TraceParams &P,
                  std::vector<double> &tables);

// True when the run needs the extended-input kernels: an energy-dependent
// rocking curve, user polarisations or further reflecting planes (the
// per-event work they change).  Source spots and user origins, directions
// and energies only change a ray's start, which every kernel takes.
bool uses_ext(const mrt_source *s, const mrt_crystal *c, const mrt_rocking_curve *r);
// Default refill threshold (lanes idle before a wave refills): for the
// plain kernels 14 in FP64 (1% faster than 12 on the von Hamos workload,
// equal on the flat one) and 12 in FP32-mixed (2-4% faster than 8), 8 for
// the extended kernels and the paper's model (2-5% faster than 12).
inline uint32_t default_refill(bool ext_or_mwg, bool f64) {
    return ext_or_mwg ? 8u : (f64 ? 14u : 12u);
}

// The paper's event model: fill its part of the parameter block (sampler
// sweeps, quadrature intervals, batch, reflection strength, density
// constants) and append the psi table to `psi`: (sin(psi_j / 2),
// psi_j - psi_{j-1}) for j = 0..M, then cos(2 psi_j) for j = 0..M.
void build_mwg_params(const mrt_crystal *c, const mrt_mosaic *m, const mrt_rocking_curve *r,
                      int burn_in, int psi_nodes, int batch, bool irc_off, TraceParams &P,
                      std::vector<double> &psi);

}  // namespace mrt
