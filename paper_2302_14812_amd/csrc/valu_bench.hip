// Issue cost of the vector instructions the deposit is made of, on one GPU: the
// rates against which its instruction mix is read (double and single
// precision arithmetic, conversions between them, and the hardware reciprocal
// and reciprocal square root seeds).
//
// Each case runs eight independent chains of one instruction per thread, in
// enough wavefronts (eight per SIMD) that latency is hidden, so the time is
// the issue cost.  Prints one JSON object: for each instruction, the cycles
// one wavefront instruction occupies a SIMD at the device's peak clock, and
// that clock.
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

constexpr int kThreads = 256;
constexpr int kChains = 8;

enum Op { kFmaF64, kAddF64, kMulF64, kFmaF32, kRsqF64, kRcpF64, kRsqF32, kRcpF32, kCvt, kNumOps };
const char* const kNames[kNumOps] = {"fma_f64", "add_f64", "mul_f64", "fma_f32", "rsq_f64",
                                     "rcp_f64", "rsq_f32", "rcp_f32", "cvt_f32_f64"};

template <int OP>
__global__ __launch_bounds__(kThreads) void chains(double* __restrict__ out, int iters, double seed)
{
    double a[kChains];
    float f[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
        a[j] = seed + threadIdx.x * 1e-3 + j;
        f[j] = (float)a[j];
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) {
            if constexpr (OP == kFmaF64)
                a[j] = fma(a[j], 0.999, 1e-3);
            else if constexpr (OP == kAddF64)
                a[j] = a[j] + 1e-3;
            else if constexpr (OP == kMulF64)
                a[j] = a[j] * 0.999;
            else if constexpr (OP == kFmaF32)
                f[j] = fmaf(f[j], 0.999f, 1e-3f);
            else if constexpr (OP == kRsqF64)
                a[j] = __builtin_amdgcn_rsq(a[j]);
            else if constexpr (OP == kRcpF64)
                a[j] = __builtin_amdgcn_rcp(a[j]);
            else if constexpr (OP == kRsqF32)
                f[j] = __builtin_amdgcn_rsqf(f[j]);
            else if constexpr (OP == kRcpF32)
                f[j] = __builtin_amdgcn_rcpf(f[j]);
            else
                a[j] = (double)(float)a[j];  // two conversions
        }
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        s += a[j] + (double)f[j];
    out[blockIdx.x * kThreads + threadIdx.x] = s;
}

template <int OP>
float time_ms(double* out, unsigned blocks, int iters)
{
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    hipLaunchKernelGGL(chains<OP>, dim3(blocks), dim3(kThreads), 0, 0, out, iters, 1.5);  // warm
    (void)hipEventRecord(e0, 0);
    hipLaunchKernelGGL(chains<OP>, dim3(blocks), dim3(kThreads), 0, 0, out, iters, 1.5);
    (void)hipEventRecord(e1, 0);
    (void)hipEventSynchronize(e1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

}  // namespace

int main()
{
    int n_cus = 0, clock_khz = 0;
    if (hipDeviceGetAttribute(&n_cus, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess ||
        hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeClockRate, 0) != hipSuccess)
        return 1;
    const int simds = 4 * n_cus;
    const unsigned blocks = (unsigned)(n_cus * 8);  // eight wavefronts per SIMD
    const int iters = 4096;
    double* out = nullptr;
    if (hipMalloc((void**)&out, (size_t)blocks * kThreads * sizeof(double)) != hipSuccess)
        return 1;
    float ms[kNumOps];
    ms[kFmaF64] = time_ms<kFmaF64>(out, blocks, iters);
    ms[kAddF64] = time_ms<kAddF64>(out, blocks, iters);
    ms[kMulF64] = time_ms<kMulF64>(out, blocks, iters);
    ms[kFmaF32] = time_ms<kFmaF32>(out, blocks, iters);
    ms[kRsqF64] = time_ms<kRsqF64>(out, blocks, iters);
    ms[kRcpF64] = time_ms<kRcpF64>(out, blocks, iters);
    ms[kRsqF32] = time_ms<kRsqF32>(out, blocks, iters);
    ms[kRcpF32] = time_ms<kRcpF32>(out, blocks, iters);
    ms[kCvt] = time_ms<kCvt>(out, blocks, iters);
    if (hipDeviceSynchronize() != hipSuccess)
        return 1;
    const double clock_hz = (double)clock_khz * 1e3;
    const double wave_instr = (double)blocks * (kThreads / 64) * iters * kChains;
    printf("{\"unit\": \"cycles per wavefront instruction per SIMD\", \"clock_ghz\": %.3f", clock_hz * 1e-9);
    for (int o = 0; o < kNumOps; ++o) {
        const double n = wave_instr * (o == kCvt ? 2.0 : 1.0);
        printf(", \"%s\": %.3f", kNames[o], (double)ms[o] * 1e-3 * clock_hz * simds / n);
    }
    printf("}\n");
    (void)hipFree(out);
    return 0;
}
