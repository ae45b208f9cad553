// VALU issue rates of gfx950 by instruction class: each kernel runs, per
// lane, 8 independent dependency chains of one instruction class for `iters`
// loop trips (4 unrolled steps of the 8 chains per trip), in enough waves
// to keep every SIMD full (32 workgroups of 4 waves per CU).
//
// The host times each launch with HIP events and reports lanes per CU per
// clock at the 2.4 GHz peak clock (what the published peaks assume), and
// each class's cost relative to v_fma_f64 (the FP64 FMA lane, one slot of
// the ALU roofline) in the same units.  The device may hold a lower clock
// under load, and not necessarily the same for every class; the relative
// costs are the ratios of measured throughputs.  Each class is timed three
// times and its best run kept.
// These rates are the slot weights of the ALU roofline of the trace kernels
// (paper_2503_16955_amd/op_costs.py).
//
// Build: hipcc -O3 --offload-arch=gfx950 -ffp-contract=off -Xclang
//        -target-feature -Xclang -packed-fp32-ops -o valu_rates valu_rates.hip
//        (no contraction: the FP32 multiply and add stay two instructions)
// Run:   ./valu_rates        (prints a markdown table)
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>

namespace {

constexpr int kChains = 8;
constexpr int kUnroll = 4;
constexpr int kOpsPerTrip = kChains * kUnroll;

enum Op { kXorAdd32, kFma32, kFma64, kMul32, kMad64, kExpLog32, kRcp32, kSqrt32, kRcp64,
          kAddMulF32, kMulHi32, kCvt32, kCmpSel32, kBitop3, kNumOps };
const char *kNames[kNumOps] = {
    "v_xor_b32 + v_add_u32 (32-bit integer ALU)", "v_fma_f32", "v_fma_f64", "v_mul_lo_u32",
    "v_mad_u64_u32", "v_exp_f32 + v_log_f32", "v_rcp_f32", "v_sqrt_f32", "v_rcp_f64",
    "v_mul_f32 + v_add_f32", "v_mul_hi_u32", "v_xor_b32 + v_cvt_f32_u32 + v_cvt_u32_f32",
    "v_cmp_gt_u32 + v_cndmask_b32", "v_bitop3_b32 (three-input XOR)"};
// VALU instructions per chain step
const int kInstPerStep[kNumOps] = {2, 1, 1, 1, 1, 2, 1, 1, 1, 2, 1, 3, 2, 1};

template <int OP>
__global__ void __launch_bounds__(256) rate_kernel(uint64_t *out, int iters, uint32_t a0,
                                                   uint32_t b0) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (OP == kXorAdd32 || OP == kMul32 || OP == kMulHi32 || OP == kCvt32 ||
                  OP == kCmpSel32 || OP == kBitop3) {
        uint32_t x[kChains];
        for (int j = 0; j < kChains; ++j) x[j] = t * 2654435761u + (uint32_t)j | 1u;
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                for (int j = 0; j < kChains; ++j) {
                    if constexpr (OP == kXorAdd32) x[j] = (x[j] ^ a0) + b0;
                    else if constexpr (OP == kMul32) x[j] = x[j] * x[j];
                    else if constexpr (OP == kMulHi32) x[j] = __umulhi(x[j], x[j]);
                    else if constexpr (OP == kCvt32) x[j] = (uint32_t)(float)(x[j] ^ a0);
                    else if constexpr (OP == kBitop3)
                        x[j] = __builtin_amdgcn_bitop3_b32(x[j], a0, x[(j + 1) % kChains], 0x96);
                    else x[j] = x[j] > a0 ? x[j] : b0;
                }
        }
        uint64_t s = 0;
        for (int j = 0; j < kChains; ++j) s += x[j];
        out[t] = s;
    } else if constexpr (OP == kMad64) {
        uint64_t x[kChains];
        for (int j = 0; j < kChains; ++j) x[j] = (uint64_t)t * 0x9E3779B97F4A7C15ull + (uint64_t)j;
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                for (int j = 0; j < kChains; ++j) x[j] = (uint64_t)(uint32_t)x[j] * a0 + x[j];
        }
        uint64_t s = 0;
        for (int j = 0; j < kChains; ++j) s += x[j];
        out[t] = s;
    } else if constexpr (OP == kFma64 || OP == kRcp64) {
        double x[kChains];
        const double m = 1.0 + (double)a0 * 1e-12, c = (double)b0 * 1e-9;
        for (int j = 0; j < kChains; ++j) x[j] = 1.0 + (double)(t + j) * 1e-7;
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                for (int j = 0; j < kChains; ++j) {
                    if constexpr (OP == kFma64) x[j] = __builtin_fma(x[j], m, c);
                    else x[j] = __builtin_amdgcn_rcp(x[j]);
                }
        }
        double s = 0.0;
        for (int j = 0; j < kChains; ++j) s += x[j];
        out[t] = (uint64_t)__double_as_longlong(s);
    } else {
        float x[kChains];
        const float m = 1.0f + (float)a0 * 1e-9f, c = (float)b0 * 1e-9f;
        for (int j = 0; j < kChains; ++j) x[j] = 1.0f + (float)(t + j) * 1e-7f;
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                for (int j = 0; j < kChains; ++j) {
                    if constexpr (OP == kFma32) x[j] = __builtin_fmaf(x[j], m, c);
                    else if constexpr (OP == kAddMulF32) x[j] = __fadd_rn(__fmul_rn(x[j], m), c);
                    else if constexpr (OP == kExpLog32)
                        x[j] = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x[j]));
                    else if constexpr (OP == kRcp32) x[j] = __builtin_amdgcn_rcpf(x[j]);
                    else x[j] = __builtin_amdgcn_sqrtf(x[j]);
                }
        }
        float s = 0.0f;
        for (int j = 0; j < kChains; ++j) s += x[j];
        out[t] = (uint64_t)__float_as_uint(s);
    }
}

// Lanes per CU per clock at the 2.4 GHz peak clock: the best of three
// timed launches (after a short warm-up launch).
template <int OP>
double measure(uint64_t *out, int blocks, int cus, int iters) {
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(256), 0, 0, out, 2, 3u, 5u);
    float best = 0.0f;
    for (int rep = 0; rep < 3; ++rep) {
        (void)hipEventRecord(e0, 0);
        hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(256), 0, 0, out, iters, 3u, 5u);
        (void)hipEventRecord(e1, 0);
        if (hipEventSynchronize(e1) != hipSuccess) {
            std::fprintf(stderr, "kernel %d failed\n", OP);
            std::exit(1);
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep == 0 || ms < best) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const double lane_inst = (double)blocks * 256.0 * iters * kOpsPerTrip * kInstPerStep[OP];
    return lane_inst / (best * 1e-3) / (cus * 2.4e9);
}

}  // namespace

int main() {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, 0) != hipSuccess) {
        std::fprintf(stderr, "no device\n");
        return 1;
    }
    const int cus = prop.multiProcessorCount;
    const int blocks = cus * 32;
    uint64_t *out = nullptr;
    if (hipMalloc(&out, sizeof(uint64_t) * blocks * 256) != hipSuccess) return 1;
    double r[kNumOps];
    r[kXorAdd32] = measure<kXorAdd32>(out, blocks, cus, 2000);
    r[kFma32] = measure<kFma32>(out, blocks, cus, 2000);
    r[kFma64] = measure<kFma64>(out, blocks, cus, 1000);
    r[kMul32] = measure<kMul32>(out, blocks, cus, 1000);
    r[kMad64] = measure<kMad64>(out, blocks, cus, 500);
    r[kExpLog32] = measure<kExpLog32>(out, blocks, cus, 500);
    r[kRcp32] = measure<kRcp32>(out, blocks, cus, 1000);
    r[kSqrt32] = measure<kSqrt32>(out, blocks, cus, 1000);
    r[kRcp64] = measure<kRcp64>(out, blocks, cus, 300);
    r[kAddMulF32] = measure<kAddMulF32>(out, blocks, cus, 1000);
    r[kMulHi32] = measure<kMulHi32>(out, blocks, cus, 1000);
    r[kCvt32] = measure<kCvt32>(out, blocks, cus, 700);
    r[kCmpSel32] = measure<kCmpSel32>(out, blocks, cus, 1000);
    r[kBitop3] = measure<kBitop3>(out, blocks, cus, 2000);
    (void)hipFree(out);
    std::printf("%s, %d CUs, peak clock %d kHz; 32 workgroups of 256 threads per CU\n\n",
                prop.gcnArchName, cus, prop.clockRate);
    std::printf("| instruction class | lanes / CU / clock at 2.4 GHz | cost relative to v_fma_f64 |\n");
    std::printf("|---|---|---|\n");
    for (int k = 0; k < kNumOps; ++k)
        std::printf("| %s | %.1f | %.2f |\n", kNames[k], r[k], r[kFma64] / r[k]);
    return 0;
}
