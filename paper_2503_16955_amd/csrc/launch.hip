// Kernel lookup across the instance translation units, the fill kernel that
// clears images and counters on the caller's stream, and the calibration map
// (mean photon energy per pixel).
#include <hip/hip_runtime.h>

#include "trace_params.h"

namespace mrt {

const void *trace_table_f64_flat(int mdf, int irc, bool rec);
const void *trace_table_f64_cyl(int mdf, int irc, bool rec);
const void *trace_table_f32_flat(int mdf, int irc, bool rec);
const void *trace_table_f32_cyl(int mdf, int irc, bool rec);

const void *ext_table_f64_flat(int mdf, int irc, bool rec);
const void *ext_table_f64_cyl(int mdf, int irc, bool rec);
const void *ext_table_f32_flat(int mdf, int irc, bool rec);
const void *ext_table_f32_cyl(int mdf, int irc, bool rec);

const void *serve_kernel_ptr_f64(bool ext);
const void *serve_kernel_ptr_f32(bool ext);

const void *serve_kernel_ptr(int precision, bool ext) {
    return precision == MRT_FP64 ? serve_kernel_ptr_f64(ext) : serve_kernel_ptr_f32(ext);
}

const void *trace_kernel_ptr(int precision, int geometry, int mdf, int irc, bool records) {
    const bool flat = geometry == MRT_GEOMETRY_FLAT;
    if (precision == MRT_FP64)
        return flat ? trace_table_f64_flat(mdf, irc, records) : trace_table_f64_cyl(mdf, irc, records);
    return flat ? trace_table_f32_flat(mdf, irc, records) : trace_table_f32_cyl(mdf, irc, records);
}

const void *ext_kernel_ptr(int precision, int geometry, int mdf, int irc, bool records) {
    const bool flat = geometry == MRT_GEOMETRY_FLAT;
    if (precision == MRT_FP64)
        return flat ? ext_table_f64_flat(mdf, irc, records) : ext_table_f64_cyl(mdf, irc, records);
    return flat ? ext_table_f32_flat(mdf, irc, records) : ext_table_f32_cyl(mdf, irc, records);
}

namespace {
__global__ void zero_kernel(uint32_t *p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// map = (energy / counts) 1e-6 keV per pixel, NaN where no photon landed
__global__ void calibration_kernel(const uint32_t *__restrict__ c,
                                   const unsigned long long *__restrict__ e, size_t n,
                                   double *__restrict__ m) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t k = c[i];
        m[i] = k ? ((double)e[i] / (double)k) * 1e-6 : __builtin_nan("");
    }
}
}  // namespace

int launch_calibration_map(const uint32_t *counts, const uint64_t *energy, size_t n, double *map,
                           void *stream) {
    if (n == 0) return 0;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(calibration_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, counts, (const unsigned long long *)energy, n, map);
    return (int)hipGetLastError();
}

int launch_zero(void *ptr, size_t n_words, void *stream) {
    if (n_words == 0) return 0;
    size_t blocks = (n_words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (uint32_t *)ptr, n_words);
    return (int)hipGetLastError();
}

}  // namespace mrt
