// Host stand-in for the device side of HIP, used to run the trace kernels'
// code on the CPU in tests: one wave is 64 coroutines (simt_emu.cpp) that
// meet at every wave-level operation (ballot, readfirstlane), so the kernels'
// SIMT control flow executes as written.  Device math builtins map to host
// functions of equal or better accuracy.
#pragma once
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <cmath>

// Every index assertion of the device loops is checked here.
void simt_check_failed(const char *cond, const char *file, int line);
#define MRT_DEV_CHECK(cond) ((cond) ? (void)0 : simt_check_failed(#cond, __FILE__, __LINE__))

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__
#define __constant__
#define MRT_CONST_AS

struct simt_dim3 {
    unsigned x, y, z;
};
extern thread_local simt_dim3 threadIdx, blockIdx, blockDim, gridDim;

// wave primitives (simt_emu.cpp)
uint64_t simt_ballot(bool p);
uint32_t simt_readfirstlane(uint32_t v);
int simt_lane();
inline void __syncthreads() {}
// wave-level memory ordering: a meeting point of the wave's lanes
inline void __builtin_amdgcn_wave_barrier() { (void)simt_readfirstlane(0); }
#define __builtin_amdgcn_fence(order, scope) ((void)0)

inline uint64_t __ballot(int p) { return simt_ballot(p != 0); }
inline int __lane_id() { return simt_lane(); }
inline unsigned long long __popcll(unsigned long long x) { return (unsigned long long)__builtin_popcountll(x); }
inline uint32_t __builtin_amdgcn_readfirstlane(uint32_t v) { return simt_readfirstlane(v); }
inline uint32_t __builtin_amdgcn_mbcnt_lo(uint32_t m, uint32_t a) {
    const int l = simt_lane();
    const uint32_t below = l >= 32 ? 0xffffffffu : ((1u << l) - 1u);
    return a + (uint32_t)__builtin_popcount(m & below);
}
inline uint32_t __builtin_amdgcn_mbcnt_hi(uint32_t m, uint32_t a) {
    const int l = simt_lane();
    const uint32_t below = l <= 32 ? 0u : ((1u << (l - 32)) - 1u);
    return a + (uint32_t)__builtin_popcount(m & below);
}

inline unsigned int atomicAdd(unsigned int *p, unsigned int v) { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }
#define __HIP_MEMORY_SCOPE_AGENT 3
template <class T> inline T __hip_atomic_load(T *p, int order, int) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
inline unsigned long long atomicAdd(unsigned long long *p, unsigned long long v) {
    return __atomic_fetch_add(p, v, __ATOMIC_RELAXED);
}

// The kernels read their by-value parameter block through this pointer; the
// emulator runs the loops below the kernels and never calls it.
inline const void *__builtin_amdgcn_kernarg_segment_ptr() { return nullptr; }

inline long long __double_as_longlong(double x) { long long r; memcpy(&r, &x, 8); return r; }
inline double __longlong_as_double(long long x) { double r; memcpy(&r, &x, 8); return r; }
inline float __uint_as_float(unsigned int x) { float r; memcpy(&r, &x, 4); return r; }
inline unsigned int __float_as_uint(float x) { unsigned int r; memcpy(&r, &x, 4); return r; }

// The hardware's FP64 reciprocal and reciprocal square root are seeds about
// 2^-24 off (v_rsq_f64 measured at 5.5e-8 relative); `simt_seed_rel` gives
// the emulated seeds that relative error, so a test can check the routines
// that refine them.
inline thread_local double simt_seed_rel = 0.0;
inline double __builtin_amdgcn_rcp(double x) { return (1.0 / x) * (1.0 + simt_seed_rel); }
// Three-input bitwise operation by truth table: result bit i is bit
// (a_i << 2 | b_i << 1 | c_i) of imm (0x96 is the three-input XOR, whose
// table does not depend on the order of the inputs).
inline uint32_t __builtin_amdgcn_bitop3_b32(uint32_t a, uint32_t b, uint32_t c, unsigned imm) {
    uint32_t r = 0;
    for (int i = 0; i < 32; ++i) {
        const unsigned idx = (((a >> i) & 1u) << 2) | (((b >> i) & 1u) << 1) | ((c >> i) & 1u);
        r |= ((imm >> idx) & 1u) << i;
    }
    return r;
}
// Funnel shift: the low 32 bits of the 64-bit (a:b) shifted right by s mod 32.
inline uint32_t __builtin_amdgcn_alignbit(uint32_t a, uint32_t b, uint32_t s) {
    return (uint32_t)(((((uint64_t)a) << 32) | b) >> (s & 31u));
}
inline double __dadd_rn(double a, double b) { return a + b; }
inline double __dsub_rn(double a, double b) { return a - b; }
inline double __dmul_rn(double a, double b) { return a * b; }
inline double __ddiv_rn(double a, double b) { return a / b; }
inline double __builtin_amdgcn_rsq(double x) { return (1.0 / std::sqrt(x)) * (1.0 + simt_seed_rel); }
// The hardware's FP32 reciprocal, square root and exp2 are within 1 ulp, not
// correctly rounded.  `simt_ulp_bias` (-1, 0, +1) moves their results one
// float toward -inf / +inf, so a test can bracket the device's answers.
inline thread_local int simt_ulp_bias = 0;
inline float simt_biased(float r) {
    if (simt_ulp_bias > 0) return std::nextafter(r, INFINITY);
    if (simt_ulp_bias < 0) return std::nextafter(r, -INFINITY);
    return r;
}
inline float __builtin_amdgcn_rcpf(float x) { return simt_biased(1.0f / x); }
inline float __builtin_amdgcn_rsqf(float x) { return 1.0f / std::sqrt(x); }
inline float __builtin_amdgcn_sqrtf(float x) { return simt_biased(std::sqrt(x)); }
inline float __builtin_amdgcn_exp2f(float x) { return simt_biased(std::exp2(x)); }
inline float __builtin_amdgcn_logf(float x) { return std::log2(x); }
inline float __builtin_amdgcn_sinf(float x) { return (float)std::sin(6.283185307179586 * (double)x); }
inline float __builtin_amdgcn_cosf(float x) { return (float)std::cos(6.283185307179586 * (double)x); }
