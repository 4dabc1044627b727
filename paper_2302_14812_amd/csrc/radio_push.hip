// The particle push of the run-time mode (Sec. 3.1: the deposit is a sub-step
// right after the push, using the new and the stored positions and momenta).
// Boris method, c = 1, u = gamma beta, in uniform fields plus a plane wave
// E = a pol cos(omega (t - k.x) + phase), B = k x E.  One step: half drift,
// the Boris kick with the fields at the half step (half electric kick,
// magnetic rotation, half electric kick), half drift; x and u stay samples at
// the same times, as the deposit reads them.  One thread per particle walks
// the steps and writes each state into the chunk arrays, so the deposit can
// read them straight from device memory.
#include "radio_internal.h"

namespace radio {

namespace {

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

__global__ __launch_bounds__(256) void boris_kernel(PushParams P, int64_t n_p, int64_t n_s,
                                                    double t_first, int64_t first_step,
                                                    double* __restrict__ x,
                                                    double* __restrict__ u)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n_p)
        return;
    const int64_t stride = (n_s + 1) * n_p;  // between components
    double xs[3], us[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        xs[k] = x[k * stride + p];
        us[k] = u[k * stride + p];
    }
    const double h = 0.5 * P.qm * P.dt;
    double kxp[3];  // k x pol, the direction of the wave's B
    cross3(P.wave_dir, P.wave_pol, kxp);
    for (int64_t s = 0; s < n_s; ++s) {
        const double g = sqrt(1.0 + (us[0] * us[0] + us[1] * us[1] + us[2] * us[2]));
        double xh[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            xh[k] = xs[k] + 0.5 * P.dt * us[k] / g;
        const double th = t_first + ((double)(first_step + s) + 0.5) * P.dt;
        double E[3], B[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            E[k] = P.E[k];
            B[k] = P.B[k];
        }
        if (P.wave_amplitude != 0.0) {
            const double ph = P.wave_omega * (th - (P.wave_dir[0] * xh[0] + P.wave_dir[1] * xh[1] +
                                                    P.wave_dir[2] * xh[2])) +
                              P.wave_phase;
            const double w = P.wave_amplitude * cos(ph);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                E[k] += w * P.wave_pol[k];
                B[k] += w * kxp[k];
            }
        }
        double um[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            um[k] = us[k] + h * E[k];
        const double gm = sqrt(1.0 + (um[0] * um[0] + um[1] * um[1] + um[2] * um[2]));
        double tv[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            tv[k] = h * B[k] / gm;
        double c1[3], up[3];
        cross3(um, tv, c1);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            up[k] = um[k] + c1[k];
        const double f = 2.0 / (1.0 + (tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2]));
        double sv[3], c2[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            sv[k] = f * tv[k];
        cross3(up, sv, c2);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            us[k] = um[k] + c2[k] + h * E[k];
        const double gn = sqrt(1.0 + (us[0] * us[0] + us[1] * us[1] + us[2] * us[2]));
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            xs[k] = xh[k] + 0.5 * P.dt * us[k] / gn;
            x[k * stride + (s + 1) * n_p + p] = xs[k];
            u[k * stride + (s + 1) * n_p + p] = us[k];
        }
    }
}

}  // namespace

hipError_t launch_push(const PushParams& P, int64_t n_p, int64_t n_s, double t_first,
                       int64_t first_step, double* x, double* u, hipStream_t s)
{
    if (n_p <= 0 || n_s <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(boris_kernel, dim3((unsigned)((n_p + 255) / 256)), dim3(256), 0, s, P,
                       n_p, n_s, t_first, first_step, x, u);
    return hipGetLastError();
}

}  // namespace radio
