// Restoring a detector from a snapshot of its fields: the inverse of the
// readout.  The detector array is the only state a deposit leaves (the
// integrator detector of Sec. 3.2 accumulates slot values, and chunks carry
// their own previous state, Sec. 3.1), so E and B as read are a complete
// checkpoint, and loading them resumes accumulation where it stopped.
#include "radio_internal.h"

namespace radio {

namespace {

// One thread per (internal row, slot): the caller's cell user_index[r] of E
// and B [n_c][n_t][3] into the accumulator [n_c][n_t][6] (double) or, for
// compensated single accumulation, the pair hi[6], lo[6] of each slot: hi the
// value rounded to single precision, lo the single-precision rounding of what
// remains (the pair then holds the value to about 2^-48 of itself).
template <bool PAIRS>
__global__ __launch_bounds__(256) void load_kernel(double* __restrict__ acc, int64_t n_c,
                                                   int64_t n_t,
                                                   const int64_t* __restrict__ user_index,
                                                   const double* __restrict__ E,
                                                   const double* __restrict__ B)
{
    const int64_t total = n_c * n_t;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / n_t;
        const int64_t j = i - r * n_t;
        const int64_t o = (user_index[r] * n_t + j) * 3;
        const double v[6] = {E[o], E[o + 1], E[o + 2], B[o], B[o + 1], B[o + 2]};
        if (PAIRS) {
            float* q = reinterpret_cast<float*>(acc) + i * 12;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const float hi = (float)v[k];
                q[k] = hi;
                q[6 + k] = (float)(v[k] - (double)hi);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 6; ++k)
                acc[i * 6 + k] = v[k];
        }
    }
}

}  // namespace

hipError_t launch_load(double* acc, int64_t n_c, int64_t n_t, const int64_t* user_index,
                       bool pairs, const double* E, const double* B, hipStream_t s)
{
    const int64_t total = n_c * n_t;
    if (total <= 0)
        return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536)
        blocks = 65536;
    if (pairs)
        hipLaunchKernelGGL(load_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, acc, n_c,
                           n_t, user_index, E, B);
    else
        hipLaunchKernelGGL(load_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, acc, n_c,
                           n_t, user_index, E, B);
    return hipGetLastError();
}

}  // namespace radio
