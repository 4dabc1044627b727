// Spectral post-processing of a detector (Sec. 4: the detector data Fourier
// transformed with respect to time, compared there with Eq. 7 and Eq. 8).
//
// A slot holds the field averaged over the slot, so the transform of the
// piecewise-constant signal at omega is
//     F(omega) = sum_j E_j e^{-i omega j dt} (e^{-i omega dt} - 1) / (-i omega)
// and, with R the cell's distance from the origin,
//     d2I/domega dOmega = c R^2 / (4 pi^2) |F(omega)|^2
//     dI/domega         = sum over cells of weight_c d2I/domega dOmega
//     dI/dOmega         = c R^2 / (4 pi) sum_j |E_j|^2 dt          (Parseval)
// at omega_m = 2 pi m / (N dt), m = 0 .. N/2, the signal zero beyond its
// n_t slots (N a power of two >= n_t).
//
// Kernels, per group of cells that fits the workspace:
//   spec_load_kernel   packs Ex + i Ey and Ez + 0i of each cell as two complex
//                      signals of length N (zero padded);
//   spec_fft_pass      one radix-2 Stockham pass (natural order in and out,
//                      no bit reversal), log2(N) launches ping-ponging
//                      between two buffers;
//   spec_power_kernel  one thread per frequency: |X|^2 + |Y|^2 of the two
//                      real signals packed in Z from Z(m) and Z(N - m),
//                      scaled to d2I, and the weighted sum over the group's
//                      cells added to dI/domega;
// and spec_parseval_kernel, one workgroup per cell, for dI/dOmega.
#include "radio_internal.h"

namespace radio {

namespace {

constexpr double kPi = 3.14159265358979323846;

template <bool PAIRS>
__global__ __launch_bounds__(256) void spec_load_kernel(const double* __restrict__ acc,
                                                        int64_t n_t, int64_t r0, int64_t G,
                                                        int64_t N, double2* __restrict__ Z)
{
    const int64_t total = G * N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = i / N;
        const int64_t j = i - g * N;
        double e[3] = {0.0, 0.0, 0.0};
        if (j < n_t) {
            const int64_t s = (r0 + g) * n_t + j;
            if (PAIRS) {
                const float* q = reinterpret_cast<const float*>(acc) + s * 12;
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    e[k] = (double)q[k] + (double)q[6 + k];
            } else {
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    e[k] = acc[s * 6 + k];
            }
        }
        Z[(2 * g) * N + j] = make_double2(e[0], e[1]);
        Z[(2 * g + 1) * N + j] = make_double2(e[2], 0.0);
    }
}

// y = one radix-2 Stockham pass of x for butterflies of span Ns, over n_sig
// signals of length N: with k = j mod Ns, x[j] and x[j + N/2] e^{-i pi k/Ns}
// combine into y[2j - k] and y[2j - k + Ns].
__global__ __launch_bounds__(256) void spec_fft_pass(const double2* __restrict__ x,
                                                     double2* __restrict__ y, int64_t N,
                                                     int64_t Ns, int64_t n_sig)
{
    const int64_t half = N / 2;
    const int64_t total = n_sig * half;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t sig = i / half;
        const int64_t j = i - sig * half;
        const double2* xs = x + sig * N;
        double2* ys = y + sig * N;
        const int64_t k = j & (Ns - 1);
        const double2 a = xs[j];
        const double2 b = xs[j + half];
        double sn, cs;
        sincospi(-(double)k / (double)Ns, &sn, &cs);
        const double2 bw = make_double2(b.x * cs - b.y * sn, b.x * sn + b.y * cs);
        const int64_t idx = 2 * j - k;  // (j / Ns) * 2 Ns + k
        ys[idx] = make_double2(a.x + bw.x, a.y + bw.y);
        ys[idx + Ns] = make_double2(a.x - bw.x, a.y - bw.y);
    }
}

__global__ __launch_bounds__(256) void spec_power_kernel(
    const double2* __restrict__ Z, int64_t N, int64_t G, int64_t r0,
    const double* __restrict__ cells, const int64_t* __restrict__ user_index,
    const double* __restrict__ weights, double dt, double c, double* __restrict__ d2I,
    double* __restrict__ dIdw, bool first_group)
{
    const int64_t n_f = N / 2 + 1;
    const int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (m >= n_f)
        return;
    const double omega = 2.0 * kPi * (double)m / ((double)N * dt);
    double W2;  // |(e^{-i w dt} - 1) / (-i w)|^2
    if (m == 0) {
        W2 = dt * dt;
    } else {
        const double s = 2.0 * sin(0.5 * omega * dt) / omega;
        W2 = s * s;
    }
    const int64_t mm = (N - m) & (N - 1);
    double sum = (first_group || !dIdw) ? 0.0 : dIdw[m];
    for (int64_t g = 0; g < G; ++g) {
        const double2* z1 = Z + (2 * g) * N;
        const double2* z2 = z1 + N;
        const double p = 0.5 * ((z1[m].x * z1[m].x + z1[m].y * z1[m].y) +
                                (z1[mm].x * z1[mm].x + z1[mm].y * z1[mm].y) +
                                (z2[m].x * z2[m].x + z2[m].y * z2[m].y) +
                                (z2[mm].x * z2[mm].x + z2[mm].y * z2[mm].y));
        const int64_t r = r0 + g;
        const double* x = cells + 3 * r;
        const double R2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        const double S = c * R2 / (4.0 * kPi * kPi) * W2 * p;
        const int64_t cell = user_index[r];
        if (d2I)
            d2I[cell * n_f + m] = S;
        sum += (weights ? weights[cell] : 1.0) * S;
    }
    if (dIdw)
        dIdw[m] = sum;
}

template <bool PAIRS>
__global__ __launch_bounds__(256) void spec_parseval_kernel(const double* __restrict__ acc,
                                                            int64_t n_t,
                                                            const double* __restrict__ cells,
                                                            const int64_t* __restrict__ user_index,
                                                            double dt, double c,
                                                            double* __restrict__ dIdO)
{
    __shared__ double part[256];
    const int64_t r = blockIdx.x;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n_t; j += 256) {
        const int64_t i = r * n_t + j;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double e;
            if (PAIRS) {
                const float* q = reinterpret_cast<const float*>(acc) + i * 12;
                e = (double)q[k] + (double)q[6 + k];
            } else {
                e = acc[i * 6 + k];
            }
            s += e * e;
        }
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double* x = cells + 3 * r;
        const double R2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        dIdO[user_index[r]] = c * R2 / (4.0 * kPi) * part[0] * dt;
    }
}

unsigned grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (unsigned)(b > 65536 ? 65536 : (b < 1 ? 1 : b));
}

}  // namespace

hipError_t launch_spectrum_group(const double* acc, bool pairs, int64_t n_t, int64_t r0,
                                 int64_t G, int64_t N, const double* cells,
                                 const int64_t* user_index, const double* weights, double dt,
                                 double c, double2* work0, double2* work1, double* d2I,
                                 double* dIdw, bool first_group, hipStream_t s)
{
    if (pairs)
        hipLaunchKernelGGL(spec_load_kernel<true>, dim3(grid_for(G * N)), dim3(256), 0, s, acc,
                           n_t, r0, G, N, work0);
    else
        hipLaunchKernelGGL(spec_load_kernel<false>, dim3(grid_for(G * N)), dim3(256), 0, s, acc,
                           n_t, r0, G, N, work0);
    double2* x = work0;
    double2* y = work1;
    for (int64_t Ns = 1; Ns < N; Ns *= 2) {
        hipLaunchKernelGGL(spec_fft_pass, dim3(grid_for(2 * G * (N / 2))), dim3(256), 0, s, x, y,
                           N, Ns, 2 * G);
        double2* t = x;
        x = y;
        y = t;
    }
    const int64_t n_f = N / 2 + 1;
    hipLaunchKernelGGL(spec_power_kernel, dim3((unsigned)((n_f + 255) / 256)), dim3(256), 0, s, x,
                       N, G, r0, cells, user_index, weights, dt, c, d2I, dIdw, first_group);
    return hipGetLastError();
}

hipError_t launch_spectrum_parseval(const double* acc, bool pairs, int64_t n_c, int64_t n_t,
                                    const double* cells, const int64_t* user_index, double dt,
                                    double c, double* dIdO, hipStream_t s)
{
    if (n_c <= 0)
        return hipSuccess;
    if (pairs)
        hipLaunchKernelGGL(spec_parseval_kernel<true>, dim3((unsigned)n_c), dim3(256), 0, s, acc,
                           n_t, cells, user_index, dt, c, dIdO);
    else
        hipLaunchKernelGGL(spec_parseval_kernel<false>, dim3((unsigned)n_c), dim3(256), 0, s,
                           acc, n_t, cells, user_index, dt, c, dIdO);
    return hipGetLastError();
}

}  // namespace radio
