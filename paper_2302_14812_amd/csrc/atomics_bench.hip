// Throughput of floating-point atomic adds on one GPU: the rates against
// which the deposit's own atomic traffic is read (ring flushes and bypasses
// go to HBM as 8-byte adds; slot emissions go to LDS rings).
//
// Cases (each thread issues `iters` adds, no return value):
//   global_f64_spread  lane i of the grid adds to element (i + k * grid) of a
//                      1 GiB array: coalesced, every line a different one
//   global_f32_spread  the same in single precision
//   global_f64_wave    all lanes of a wavefront add to one element (a
//                      different element per wavefront): contended
//   lds_f64_spread     lane i adds to LDS element i (no bank conflicts)
//   lds_f64_wave       all lanes of a wavefront add to one LDS element
// Prints one JSON object: atomic adds per second per case.
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

constexpr int kThreads = 256;

template <typename T>
__global__ __launch_bounds__(kThreads) void global_spread(T* __restrict__ buf, int64_t n,
                                                           int iters)
{
    const int64_t grid = (int64_t)gridDim.x * blockDim.x;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int k = 0; k < iters; ++k) {
        const int64_t j = (i + (int64_t)k * grid) % n;
        unsafeAtomicAdd(buf + j, T(1));
    }
}

__global__ __launch_bounds__(kThreads) void global_wave(double* __restrict__ buf, int64_t n,
                                                        int iters)
{
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / 64;
    for (int k = 0; k < iters; ++k)
        unsafeAtomicAdd(buf + (wave * 8 + k) % n, 1.0);
}

template <bool WAVE>
__global__ __launch_bounds__(kThreads) void lds_add(double* __restrict__ out, int iters)
{
    __shared__ double s[kThreads];
    s[threadIdx.x] = 0.0;
    __syncthreads();
    const int slot = WAVE ? (int)(threadIdx.x / 64) : (int)threadIdx.x;
    for (int k = 0; k < iters; ++k)
        __hip_atomic_fetch_add(s + slot, 1.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();
    if (threadIdx.x == 0)
        out[blockIdx.x] = s[0];
}

template <typename F>
double time_ms(F launch)
{
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    launch();  // warm
    (void)hipEventRecord(a, 0);
    launch();
    (void)hipEventRecord(b, 0);
    (void)hipEventSynchronize(b);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return (double)ms;
}

}  // namespace

int main()
{
    int n_cus = 0;
    if (hipDeviceGetAttribute(&n_cus, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess)
        return 1;
    const int64_t bytes = (int64_t)1 << 30;
    void* buf = nullptr;
    double* out = nullptr;
    const unsigned blocks = (unsigned)(n_cus * 8);
    if (hipMalloc(&buf, bytes) != hipSuccess || hipMalloc((void**)&out, blocks * sizeof(double)) != hipSuccess)
        return 1;
    if (hipMemset(buf, 0, bytes) != hipSuccess)
        return 1;
    const int64_t n64 = bytes / 8, n32 = bytes / 4;
    const int it_g = 64, it_l = 4096;
    const double adds_g = (double)blocks * kThreads * it_g;
    const double adds_l = (double)blocks * kThreads * it_l;
    const double g64 = time_ms([&] {
        hipLaunchKernelGGL(global_spread<double>, dim3(blocks), dim3(kThreads), 0, 0, (double*)buf, n64, it_g);
    });
    const double g32 = time_ms([&] {
        hipLaunchKernelGGL(global_spread<float>, dim3(blocks), dim3(kThreads), 0, 0, (float*)buf, n32, it_g);
    });
    const double gw = time_ms([&] {
        hipLaunchKernelGGL(global_wave, dim3(blocks), dim3(kThreads), 0, 0, (double*)buf, n64, it_g);
    });
    const double ls = time_ms([&] {
        hipLaunchKernelGGL(lds_add<false>, dim3(blocks), dim3(kThreads), 0, 0, out, it_l);
    });
    const double lw = time_ms([&] {
        hipLaunchKernelGGL(lds_add<true>, dim3(blocks), dim3(kThreads), 0, 0, out, it_l);
    });
    if (hipDeviceSynchronize() != hipSuccess)
        return 1;
    printf("{\"unit\": \"atomic adds/s\", \"global_f64_spread\": %.4e, \"global_f32_spread\": %.4e, "
           "\"global_f64_wave\": %.4e, \"lds_f64_spread\": %.4e, \"lds_f64_wave\": %.4e}\n",
           adds_g / (g64 * 1e-3), adds_g / (g32 * 1e-3), adds_g / (gw * 1e-3), adds_l / (ls * 1e-3),
           adds_l / (lw * 1e-3));
    (void)hipFree(buf);
    (void)hipFree(out);
    return 0;
}
