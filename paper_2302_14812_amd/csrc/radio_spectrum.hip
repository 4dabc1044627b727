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
// Each cell gives two complex signals of length N (zero padded): Z1 = Ex + i Ey
// and Z2 = Ez + 0i.  The power of the three real components at omega_m is
// (Q(m) + Q(N - m)) / 2 with Q(m) = |Z1(m)|^2 + |Z2(m)|^2.  Kernels, per group
// of cells that fits the workspace:
//   spec_cols_kernel   (N = N1 * N2, N1 and N2 <= kFftTile) the first of the
//                      two steps of the four-step FFT: with n = N2 n1 + n2,
//                      tiles of columns (fixed n2, n1 = 0 .. N1 - 1) are read
//                      from the detector, transformed in LDS, multiplied by
//                      exp(-2 pi i n2 k1 / N) and stored at N2 k1 + n2;
//                      spec_cols2_kernel does the same for both signals of a
//                      cell in one tile, so that each slot is read once;
//   spec_rows_kernel   the second step: tiles of rows (fixed k1, contiguous)
//                      transformed in LDS and stored at k1 + N1 k2, the
//                      spectrum in natural order; spec_rows_q_kernel
//                      transforms the rows of both signals of a cell together
//                      and stores only Q, row-major (8 bytes a frequency
//                      instead of 32);
//                      For N <= kFftTile the first step alone is the transform
//                      (N2 = 1);
//   spec_load_kernel + spec_fft_pass   for N > kFftTile^2: packing, then
//                      log2(N) radix-2 Stockham passes between two buffers;
//   spec_power_kernel  a thread per frequency and block of cells: the power
//                      from Z1 and Z2 at m and N - m, scaled to d2I, and the
//                      weighted sum over its cells added to dI/domega
//                      (atomically); spec_power_t_kernel does the same from
//                      the row-major Q, transposing tiles through LDS;
// and spec_parseval_kernel, one workgroup per cell, for dI/dOmega.
#include <algorithm>

#include "radio_internal.h"

namespace radio {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kFftTileLg = 11;
constexpr int kFftTile = 1 << kFftTileLg;  // complex values transformed per workgroup in LDS
constexpr int kFftThreads = 256;

// value n (< N) of signal s (2 g: Ex + i Ey of cell r0 + g; 2 g + 1: Ez) of the
// detector's accumulator; zero past its n_t slots
template <bool PAIRS>
__device__ __forceinline__ double2 signal_at(const double* __restrict__ acc, int64_t n_t,
                                             int64_t r0, int64_t s, int64_t n)
{
    if (n >= n_t)
        return make_double2(0.0, 0.0);
    const int64_t i = (r0 + (s >> 1)) * n_t + n;
    double e[3];
    if (PAIRS) {
        const float* q = reinterpret_cast<const float*>(acc) + i * 12;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            e[k] = (double)q[k] + (double)q[6 + k];
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k)
            e[k] = acc[i * 6 + k];
    }
    return (s & 1) ? make_double2(e[2], 0.0) : make_double2(e[0], e[1]);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Twiddle tables of a transform of N = 2^lg (lg <= 2 kFftTileLg), written by
// spec_tables_kernel into kSpecTableValues complex values:
//   tab[k]          = exp(-2 pi i k / kFftTile), k < kFftTile / 2: an LDS
//                     transform of length len <= kFftTile takes every
//                     (kFftTile / len)-th entry;
//   tab[kTabLo + b] = exp(-2 pi i b / N), b < S = 2^ceil(lg / 2);
//   tab[kTabHi + a] = exp(-2 pi i a S / N), a < N / S;
// so that exp(-2 pi i r / N) = tab[kTabHi + r / S] tab[kTabLo + r mod S].
constexpr int kTabLo = kFftTile / 2;
constexpr int kTabHi = kTabLo + kFftTile;
static_assert(kTabHi + kFftTile <= kSpecTableValues, "twiddle table layout");

__global__ __launch_bounds__(256) void spec_tables_kernel(double2* __restrict__ tab, int lg)
{
    const int lgS = (lg + 1) / 2;
    const int64_t N = (int64_t)1 << lg;
    const int S = 1 << lgS;
    const int A = (int)(N >> lgS);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < (int)kSpecTableValues;
         i += gridDim.x * blockDim.x) {
        double x;  // the angle in units of -2 pi
        if (i < kTabLo)
            x = (double)i / (double)kFftTile;
        else if (i < kTabLo + S)
            x = (double)(i - kTabLo) / (double)N;
        else if (i >= kTabHi && i < kTabHi + A)
            x = (double)((int64_t)(i - kTabHi) << lgS) / (double)N;
        else
            continue;
        double sn, cs;
        sincospi(-2.0 * x, &sn, &cs);
        tab[i] = make_double2(cs, sn);
    }
}

// exp(-2 pi i r / N) for 0 <= r < N, lgS = ceil(log2(N) / 2)
__device__ __forceinline__ double2 twiddle(const double2* __restrict__ tab, int64_t r, int lgS)
{
    return cmul(tab[kTabHi + (r >> lgS)], tab[kTabLo + (r & (((int64_t)1 << lgS) - 1))]);
}

// exp(-2 pi i k / len) for k = 0 .. len/2 - 1 (len = 2^lg <= kFftTile), into tw
__device__ __forceinline__ void fill_twiddles(double2* tw, const double2* __restrict__ tab, int lg)
{
    for (int k = threadIdx.x; k < (1 << lg) / 2; k += blockDim.x)
        tw[k] = tab[k << (kFftTileLg - lg)];
}

// In-place radix-2 transform (decimation in time) of T sequences of length
// len = 2^lg in LDS, sequence t at buf[t * len], loaded in bit-reversed order;
// leaves them in natural order.  Two consecutive stages (spans h and 2h) are
// done per pass on the four values k, k + h, k + 2h, k + 3h of each block of
// 4h -- the same butterflies as two radix-2 stages, with half the passes,
// barriers and LDS traffic; an odd lg starts with one stage of span 1.  tw holds
// exp(-2 pi i j / len), j < len / 2; a pass reads one twiddle per butterfly
// and derives the other two.  Ends with a barrier.
__device__ __forceinline__ void lds_fft(double2* buf, const double2* tw, int lg, int T)
{
    const int len = 1 << lg;
    const int halfn = len >> 1;
    int lgh = 0;
    if (lg & 1) {
        __syncthreads();
        for (int b = threadIdx.x; b < T * halfn; b += blockDim.x) {
            double2* x = buf + 2 * b;
            const double2 a = x[0], c = x[1];
            x[0] = make_double2(a.x + c.x, a.y + c.y);
            x[1] = make_double2(a.x - c.x, a.y - c.y);
        }
        lgh = 1;
    }
    for (; lgh + 2 <= lg; lgh += 2) {
        __syncthreads();
        const int h = 1 << lgh;
        const int tws = halfn >> lgh;  // W_2h^k = tw[k tws], W_4h^k = tw[k tws / 2]
        for (int b = threadIdx.x; b < T * (len >> 2); b += blockDim.x) {
            const int k = b & (h - 1);
            double2* x = buf + ((b >> lgh) << (lgh + 2)) + k;
            const double2 a0 = x[0], a1 = x[h], a2 = x[2 * h], a3 = x[3 * h];
            // W_4h^k from the table; W_2h^k = (W_4h^k)^2 and W_4h^(k+h) = -i W_4h^k
            const double2 w2 = tw[k * (tws >> 1)];
            const double2 w1 = cmul(w2, w2);
            const double2 w3 = make_double2(w2.y, -w2.x);
            const double2 t1 = cmul(a1, w1), t3 = cmul(a3, w1);
            const double2 b0 = make_double2(a0.x + t1.x, a0.y + t1.y);
            const double2 b1 = make_double2(a0.x - t1.x, a0.y - t1.y);
            const double2 b2 = make_double2(a2.x + t3.x, a2.y + t3.y);
            const double2 b3 = make_double2(a2.x - t3.x, a2.y - t3.y);
            const double2 t2 = cmul(b2, w2), t4 = cmul(b3, w3);
            x[0] = make_double2(b0.x + t2.x, b0.y + t2.y);
            x[2 * h] = make_double2(b0.x - t2.x, b0.y - t2.y);
            x[h] = make_double2(b1.x + t4.x, b1.y + t4.y);
            x[3 * h] = make_double2(b1.x - t4.x, b1.y - t4.y);
        }
    }
    __syncthreads();
}

__device__ __forceinline__ int bitrev(int v, int lg)
{
    return lg == 0 ? 0 : (int)(__builtin_bitreverse32((unsigned)v) >> (32 - lg));
}

// First step: tile = T columns c (c = s * N2 + n2 over the group's 2 G signals)
// of N1 = 2^lg1 values each.  Output Y[s][N2 k1 + n2] = twiddled column FFTs.
template <bool PAIRS>
__global__ __launch_bounds__(kFftThreads) void spec_cols_kernel(const double* __restrict__ acc,
                                                                 int64_t n_t, int64_t r0,
                                                                 int64_t n_sig, int lg1, int lg2,
                                                                 const double2* __restrict__ tab,
                                                                 double2* __restrict__ Y)
{
    extern __shared__ double2 lds[];
    const int N1 = 1 << lg1;
    const int64_t N2 = (int64_t)1 << lg2;
    const int64_t N = (int64_t)N1 * N2;
    const int lgT = kFftTileLg - lg1;  // lg1 <= kFftTileLg
    const int T = 1 << lgT;             // columns per tile
    double2* buf = lds;
    double2* tw = lds + T * N1;
    const int64_t c0 = (int64_t)blockIdx.x * T;
    const int64_t n_cols = n_sig * N2;
    const int lgS = (lg1 + lg2 + 1) / 2;
    fill_twiddles(tw, tab, lg1);
    // load: consecutive threads take consecutive columns of one row n1
    for (int e = threadIdx.x; e < T * N1; e += blockDim.x) {
        const int n1 = e >> lgT;
        const int t = e & (T - 1);
        const int64_t c = c0 + t;
        double2 v = make_double2(0.0, 0.0);
        if (c < n_cols) {
            const int64_t sg = c >> lg2;
            const int64_t n2 = c & (N2 - 1);
            v = signal_at<PAIRS>(acc, n_t, r0, sg, N2 * n1 + n2);
        }
        buf[t * N1 + bitrev(n1, lg1)] = v;
    }
    lds_fft(buf, tw, lg1, T);
    for (int e = threadIdx.x; e < T * N1; e += blockDim.x) {
        const int k1 = e >> lgT;
        const int t = e & (T - 1);
        const int64_t c = c0 + t;
        if (c >= n_cols)
            continue;
        const int64_t sg = c >> lg2;
        const int64_t n2 = c & (N2 - 1);
        double2 v = buf[t * N1 + k1];
        if (lg2 > 0)  // exp(-2 pi i n2 k1 / N), argument reduced exactly
            v = cmul(v, twiddle(tab, (n2 * (int64_t)k1) & (N - 1), lgS));
        Y[sg * N + N2 * k1 + n2] = v;
    }
}

// Second step: tile = R rows (k1) of N2 = 2^lg2 contiguous values of one
// signal; X[s][k1 + N1 k2] = FFT over n2 of Y[s][N2 k1 + n2].
__global__ __launch_bounds__(kFftThreads) void spec_rows_kernel(const double2* __restrict__ Y,
                                                                 int64_t n_sig, int lg1, int lg2,
                                                                 const double2* __restrict__ tab,
                                                                 double2* __restrict__ X)
{
    extern __shared__ double2 lds[];
    const int64_t N1 = (int64_t)1 << lg1;
    const int N2 = 1 << lg2;
    const int64_t N = N1 * N2;
    const int lgR = kFftTileLg - lg2;  // lg2 <= kFftTileLg <= lg1 + lg2
    const int R = 1 << lgR;             // rows per tile (N1 is a multiple of R)
    double2* buf = lds;
    double2* tw = lds + R * N2;
    const int64_t tiles_per_sig = N1 / R;
    const int64_t sg = blockIdx.x / tiles_per_sig;
    const int64_t k10 = (blockIdx.x - sg * tiles_per_sig) * R;
    if (sg >= n_sig)
        return;
    fill_twiddles(tw, tab, lg2);
    const double2* y = Y + sg * N + N2 * k10;  // R contiguous rows
    for (int e = threadIdx.x; e < R * N2; e += blockDim.x) {
        const int r = e >> lg2;
        const int n2 = e & (N2 - 1);
        buf[r * N2 + bitrev(n2, lg2)] = y[e];
    }
    lds_fft(buf, tw, lg2, R);
    // store: consecutive threads take consecutive rows of one k2
    double2* x = X + sg * N + k10;
    for (int e = threadIdx.x; e < R * N2; e += blockDim.x) {
        const int k2 = e >> lgR;
        const int r = e & (R - 1);
        x[N1 * k2 + r] = buf[r * N2 + k2];
    }
}

// First step for both signals of cell g at once: tile = Tc consecutive columns
// n2 (Tc = kFftTile / (2 N1), so lg1 < kFftTileLg; N2 is a multiple of Tc),
// buf[s][tc][N1] for signal s = 0 (Ex + i Ey) and 1 (Ez).  Each slot of the
// detector is read once; the twiddle is shared by the two signals.  With part
// set, the tile also leaves the sum of |E|^2 over its slots in
// part[g][tile] (Parseval, reduced per cell by spec_parseval_parts_kernel).
template <bool PAIRS>
__global__ __launch_bounds__(kFftThreads) void spec_cols2_kernel(const double* __restrict__ acc,
                                                                  int64_t n_t, int64_t r0,
                                                                  int64_t G, int lg1, int lg2,
                                                                  const double2* __restrict__ tab,
                                                                  double2* __restrict__ Y,
                                                                  double* __restrict__ part)
{
    __shared__ double red[kFftThreads];
    extern __shared__ double2 lds[];
    const int N1 = 1 << lg1;
    const int64_t N2 = (int64_t)1 << lg2;
    const int64_t N = (int64_t)N1 * N2;
    const int lgTc = kFftTileLg - 1 - lg1;
    const int Tc = 1 << lgTc;
    double2* buf = lds;
    double2* tw = lds + 2 * Tc * N1;
    const int64_t tiles_per_cell = N2 >> lgTc;
    const int64_t g = blockIdx.x / tiles_per_cell;
    const int64_t n20 = (blockIdx.x - g * tiles_per_cell) << lgTc;
    if (g >= G)
        return;
    const int lgS = (lg1 + lg2 + 1) / 2;
    fill_twiddles(tw, tab, lg1);
    // load: consecutive threads take consecutive columns (slots) of one row n1
    double e2 = 0.0;
    for (int e = threadIdx.x; e < Tc * N1; e += blockDim.x) {
        const int n1 = e >> lgTc;
        const int tc = e & (Tc - 1);
        const int j = bitrev(n1, lg1);
        const double2 v0 = signal_at<PAIRS>(acc, n_t, r0, 2 * g, N2 * n1 + n20 + tc);
        const double2 v1 = signal_at<PAIRS>(acc, n_t, r0, 2 * g + 1, N2 * n1 + n20 + tc);
        buf[tc * N1 + j] = v0;
        buf[(Tc + tc) * N1 + j] = v1;
        e2 += (v0.x * v0.x + v0.y * v0.y) + v1.x * v1.x;
    }
    if (part) {
        red[threadIdx.x] = e2;
        for (int w = kFftThreads / 2; w > 0; w >>= 1) {
            __syncthreads();
            if ((int)threadIdx.x < w)
                red[threadIdx.x] += red[threadIdx.x + w];
        }
        if (threadIdx.x == 0)
            part[blockIdx.x] = red[0];
    }
    lds_fft(buf, tw, lg1, 2 * Tc);
    double2* y1 = Y + (2 * g) * N;
    double2* y2 = y1 + N;
    for (int e = threadIdx.x; e < Tc * N1; e += blockDim.x) {
        const int k1 = e >> lgTc;
        const int tc = e & (Tc - 1);
        const int64_t n2 = n20 + tc;
        // exp(-2 pi i n2 k1 / N), argument reduced exactly
        const double2 w = twiddle(tab, (n2 * (int64_t)k1) & (N - 1), lgS);
        y1[N2 * k1 + n2] = cmul(buf[tc * N1 + k1], w);
        y2[N2 * k1 + n2] = cmul(buf[(Tc + tc) * N1 + k1], w);
    }
}

// Second step for both signals of cell g, folding the two transforms into Q:
// tile = Rh rows k1 of each signal (Rh = kFftTile / (2 N2), so lg2 <
// kFftTileLg; N1 is a multiple of Rh), buf[s][r][N2].  Q is stored row-major,
// Qt[g][k1 N2 + k2] = |Z1|^2 + |Z2|^2 at frequency k1 + N1 k2, so that the
// stores are contiguous; spec_power_t_kernel transposes it.
__global__ __launch_bounds__(kFftThreads) void spec_rows_q_kernel(const double2* __restrict__ Y,
                                                                   int64_t G, int lg1, int lg2,
                                                                   const double2* __restrict__ tab,
                                                                   double* __restrict__ Q)
{
    extern __shared__ double2 lds[];
    const int64_t N1 = (int64_t)1 << lg1;
    const int N2 = 1 << lg2;
    const int64_t N = N1 * N2;
    const int lgH = kFftTileLg - 1 - lg2;
    const int Rh = 1 << lgH;
    double2* buf = lds;
    double2* tw = lds + 2 * Rh * N2;
    const int64_t tiles_per_cell = N1 >> lgH;
    const int64_t g = blockIdx.x / tiles_per_cell;
    const int64_t k10 = (blockIdx.x - g * tiles_per_cell) << lgH;
    if (g >= G)
        return;
    fill_twiddles(tw, tab, lg2);
    const double2* y = Y + (2 * g) * N + N2 * k10;  // Rh contiguous rows of signal 0
    for (int e = threadIdx.x; e < Rh * N2; e += blockDim.x) {
        const int r = e >> lg2;
        const int j = bitrev(e & (N2 - 1), lg2);
        buf[r * N2 + j] = y[e];
        buf[(Rh + r) * N2 + j] = y[N + e];
    }
    lds_fft(buf, tw, lg2, 2 * Rh);
    double* q = Q + g * N + N2 * k10;  // Rh contiguous rows
    for (int e = threadIdx.x; e < Rh * N2; e += blockDim.x) {
        const double2 a = buf[e];
        const double2 b = buf[Rh * N2 + e];
        q[e] = (a.x * a.x + a.y * a.y) + (b.x * b.x + b.y * b.y);
    }
}

// In-register radix-2 transform (decimation in time) of 2^LG values loaded in
// bit-reversed order, leaving them in natural order.  W[j] = exp(-2 pi i j /
// 2^LG), j < 2^(LG-1), read with uniform addresses (scalar loads: the same
// twiddles for every lane); the j = 0 butterflies take no product.
template <int LG>
__device__ __forceinline__ void reg_fft(double2 (&v)[1 << LG], const double2* __restrict__ W)
{
#pragma unroll
    for (int s = 0; s < LG; ++s) {
        const int h = 1 << s;
#pragma unroll
        for (int j = 0; j < h; ++j) {
            const double2 w = j == 0 ? make_double2(1.0, 0.0) : W[j << (LG - 1 - s)];
#pragma unroll
            for (int blk = 0; blk < (1 << LG); blk += 2 * h) {
                const double2 a = v[blk + j];
                const double2 t = j == 0 ? v[blk + j + h] : cmul(v[blk + j + h], w);
                v[blk + j] = make_double2(a.x + t.x, a.y + t.y);
                v[blk + j + h] = make_double2(a.x - t.x, a.y - t.y);
            }
        }
    }
}

constexpr int kRow32 = 32;  // N2 = 1024 = 32 x 32

// The second step for rows of N2 = 1024, held in registers instead of LDS
// passes: a row is a 32 x 32 four-step transform (n = 32 a + b, k = c + 32 d),
//     X[c + 32 d] = sum_b W_32^(b d) W_1024^(b c) sum_a x[32 a + b] W_32^(a c).
// One wavefront per row k1 of a cell: lanes 0-31 take signal Z1, lanes 32-63
// signal Z2.  Lane b loads x[32 a + b] (a = 0 .. 31, coalesced over the lanes),
// transforms over a in registers, multiplies by W_1024^(b c) and writes the 32
// values to LDS; lane c then reads A[b][c] (b = 0 .. 31) and transforms over b.
// Q = |Z1|^2 + |Z2|^2 is folded through LDS and stored row-major at
// Qt[g][1024 k1 + c + 32 d], as spec_rows_q_kernel stores it.
__global__ __launch_bounds__(64) void spec_rows_q32_kernel(const double2* __restrict__ Y,
                                                           int64_t G, int lg1,
                                                           const double2* __restrict__ tab,
                                                           double* __restrict__ Q)
{
    __shared__ double2 T[2][kRow32][kRow32 + 1];  // A[b][c] per signal, rows padded
    const int lane = threadIdx.x;
    const int sig = lane >> 5;
    const int b = lane & (kRow32 - 1);
    const int64_t N1 = (int64_t)1 << lg1;
    const int64_t N = N1 * (kRow32 * kRow32);
    const int64_t g = blockIdx.x >> lg1;
    const int64_t k1 = blockIdx.x & (N1 - 1);
    if (g >= G)
        return;
    // exp(-2 pi i j / 32) = tab[64 j] (tab[k] = exp(-2 pi i k / kFftTile))
    static_assert(kFftTile == 64 * kRow32, "32-point twiddles from the LDS-transform table");
    double2 w32[kRow32 / 2];
#pragma unroll
    for (int j = 0; j < kRow32 / 2; ++j)
        w32[j] = tab[64 * j];
    const double2* y = Y + (2 * g + sig) * N + (kRow32 * kRow32) * k1;
    double2 v[kRow32];
#pragma unroll
    for (int a = 0; a < kRow32; ++a)
        v[bitrev(a, 5)] = y[kRow32 * a + b];
    reg_fft<5>(v, w32);
#pragma unroll
    for (int c = 0; c < kRow32; ++c) {
        // W_1024^m = tab[2 m] for m < 512, -tab[2 m - 1024] above
        const int m = (b * c) & 1023;
        const double2 t = tab[(2 * m) & 1023];
        const double2 w = m < 512 ? t : make_double2(-t.x, -t.y);
        T[sig][c][b] = c == 0 ? v[0] : cmul(v[c], w);
    }
    __syncthreads();
#pragma unroll
    for (int bb = 0; bb < kRow32; ++bb)
        v[bitrev(bb, 5)] = T[sig][b][bb];
    reg_fft<5>(v, w32);
    __syncthreads();  // T is reused for |Z2|^2
    double* P = reinterpret_cast<double*>(&T[0][0][0]);  // [32][33] doubles
    if (sig == 1) {
#pragma unroll
        for (int d = 0; d < kRow32; ++d)
            P[d * (kRow32 + 1) + b] = v[d].x * v[d].x + v[d].y * v[d].y;
    }
    __syncthreads();
    if (sig == 0) {
        double* q = Q + g * N + (kRow32 * kRow32) * k1;
#pragma unroll
        for (int d = 0; d < kRow32; ++d)
            q[b + kRow32 * d] = (v[d].x * v[d].x + v[d].y * v[d].y) + P[d * (kRow32 + 1) + b];
    }
}

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

// d2I of kPowerCells cells of the group per thread, one thread per frequency
// m of a block, from Z1, Z2 of cell g (at Z[2g], Z[2g+1], natural order);
// their weighted sum is added to dIdw[m] (zeroed beforehand)
constexpr int kPowerCells = 16;

__global__ __launch_bounds__(256) void spec_power_kernel(
    const double2* __restrict__ Z, int64_t N, int64_t G, int64_t r0,
    const double* __restrict__ cells, const int64_t* __restrict__ user_index,
    const double* __restrict__ weights, double dt, double c, double* __restrict__ d2I,
    double* __restrict__ dIdw)
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
    double sum = 0.0;
    const int64_t g0 = (int64_t)blockIdx.y * kPowerCells;
    const int64_t g1 = g0 + kPowerCells < G ? g0 + kPowerCells : G;
    for (int64_t g = g0; g < g1; ++g) {
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
        unsafeAtomicAdd(dIdw + m, sum);
}

// Power spectra from Qt (row-major Q of spec_rows_q_kernel, N1 = 2^lg1 rows of
// N2 = 2^lg2 with lg1 + lg2 = log2 N, lg2 >= 5): a workgroup takes a tile of
// B1 = min(N1, 32) consecutive k1 by B2 = kPowerTile / B1 consecutive k2 and
// transposes it through LDS, so that its reads (along k2, both Q(m) and
// Q(N - m)) and its d2I stores (along m = k1 + N1 k2) are contiguous.  Tiles
// cover k2 <= N2 / 2, i.e. m <= N / 2; kPowerCells cells per workgroup, whose
// weighted sum is added to dIdw[m] (zeroed beforehand).
constexpr int kPowerTileLg = 10;
constexpr int kPowerTile = 1 << kPowerTileLg;

__global__ __launch_bounds__(256) void spec_power_t_kernel(
    const double* __restrict__ Qt, int lg1, int lg2, int64_t G, int64_t r0,
    const double* __restrict__ cells, const int64_t* __restrict__ user_index,
    const double* __restrict__ weights, double dt, double c, double* __restrict__ d2I,
    double* __restrict__ dIdw)
{
    constexpr int kPer = kPowerTile / 256;  // tile values per thread
    const int lgB1 = lg1 < 5 ? lg1 : 5;
    const int B1 = 1 << lgB1;
    const int lgB2 = kPowerTileLg - lgB1;
    const int B2 = 1 << lgB2;
    const int stride = B2 + 1;  // LDS row of one k1, padded
    __shared__ double tile[kPowerTile + 32];
    const int64_t N1 = (int64_t)1 << lg1, N2 = (int64_t)1 << lg2;
    const int64_t N = N1 * N2;
    const int64_t n_f = N / 2 + 1;
    const int64_t tiles1 = N1 >> lgB1;
    const int64_t k1_0 = (int64_t)(blockIdx.x % tiles1) << lgB1;
    const int64_t k2_0 = (int64_t)(blockIdx.x / tiles1) << lgB2;
    // the thread's store slots: m and the slot weight |(e^{-i w dt} - 1)/(-i w)|^2
    int64_t mo[kPer];
    double W2[kPer], sum[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int e = threadIdx.x + 256 * i;
        const int64_t m = (k1_0 + (e & (B1 - 1))) + N1 * (k2_0 + (e >> lgB1));
        mo[i] = m < n_f ? m : -1;
        const double omega = 2.0 * kPi * (double)m / ((double)N * dt);
        const double sw = m == 0 ? dt : 2.0 * sin(0.5 * omega * dt) / omega;
        W2[i] = sw * sw;
        sum[i] = 0.0;
    }
    const int64_t g0 = (int64_t)blockIdx.y * kPowerCells;
    const int64_t g1 = g0 + kPowerCells < G ? g0 + kPowerCells : G;
    for (int64_t g = g0; g < g1; ++g) {
        const double* q = Qt + g * N;
        // load along k2: Q(m) and Q(N - m), m = k1 + N1 k2 (k2 < N2 / 2 + B2 <= N2)
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + 256 * i;
            const int k1l = e >> lgB2, k2l = e & (B2 - 1);
            const int64_t k1 = k1_0 + k1l, k2 = k2_0 + k2l;
            const int64_t k1m = (N1 - k1) & (N1 - 1);
            const int64_t k2m = k1 == 0 ? (N2 - k2) & (N2 - 1) : N2 - 1 - k2;
            tile[k1l * stride + k2l] = 0.5 * (q[k1 * N2 + k2] + q[k1m * N2 + k2m]);
        }
        __syncthreads();
        const int64_t r = r0 + g;
        const double* x = cells + 3 * r;
        const double R2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        const double scale = c * R2 / (4.0 * kPi * kPi);
        const int64_t cell = user_index[r];
        const double wc = weights ? weights[cell] : 1.0;
        // store along m
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            if (mo[i] < 0)
                continue;
            const int e = threadIdx.x + 256 * i;
            const double S = scale * W2[i] * tile[(e & (B1 - 1)) * stride + (e >> lgB1)];
            if (d2I)
                d2I[cell * n_f + mo[i]] = S;
            sum[i] += wc * S;
        }
        __syncthreads();  // the tile is refilled for the next cell
    }
    if (dIdw) {
#pragma unroll
        for (int i = 0; i < kPer; ++i)
            if (mo[i] >= 0)
                unsafeAtomicAdd(dIdw + mo[i], sum[i]);
    }
}

__global__ __launch_bounds__(256) void spec_zero_kernel(double* __restrict__ p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
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

// dI/dOmega of the cells of a group from the per-tile sums of |E|^2 left by
// spec_cols2_kernel (part[g][0 .. tiles_per_cell), added in order)
__global__ __launch_bounds__(256) void spec_parseval_parts_kernel(
    const double* __restrict__ part, int64_t tiles_per_cell, int64_t G, int64_t r0,
    const double* __restrict__ cells, const int64_t* __restrict__ user_index, double dt, double c,
    double* __restrict__ dIdO)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= G)
        return;
    double sum = 0.0;
    for (int64_t i = 0; i < tiles_per_cell; ++i)
        sum += part[g * tiles_per_cell + i];
    const int64_t r = r0 + g;
    const double* x = cells + 3 * r;
    const double R2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    dIdO[user_index[r]] = c * R2 / (4.0 * kPi) * sum * dt;
}

unsigned grid_for(int64_t n);

// power spectra of a group from its transforms Z in natural order, or from
// the row-major Qt of the rows step (lg_q1 = log2 N1 > 0); dIdw is zeroed
// before the first group adds to it
hipError_t launch_power(const double2* Z, int lg_q1, int64_t N, int64_t G, int64_t r0,
                        const double* cells, const int64_t* user_index, const double* weights,
                        double dt, double c, double* d2I, double* dIdw, bool first_group,
                        hipStream_t s)
{
    const int64_t n_f = N / 2 + 1;
    if (dIdw && first_group)
        hipLaunchKernelGGL(spec_zero_kernel, dim3(grid_for(n_f)), dim3(256), 0, s, dIdw, n_f);
    const unsigned grid_y = (unsigned)((G + kPowerCells - 1) / kPowerCells);
    if (lg_q1 > 0) {
        int lg = 0;
        while (((int64_t)1 << lg) < N)
            ++lg;
        const int lg2 = lg - lg_q1;
        const int lgB1 = lg_q1 < 5 ? lg_q1 : 5;
        const int64_t B2 = (int64_t)1 << (kPowerTileLg - lgB1);
        const int64_t tiles2 = (((int64_t)1 << lg2) / 2 + 1 + B2 - 1) / B2;
        const int64_t tiles1 = ((int64_t)1 << lg_q1) >> lgB1;
        hipLaunchKernelGGL(spec_power_t_kernel, dim3((unsigned)(tiles1 * tiles2), grid_y),
                           dim3(256), 0, s, reinterpret_cast<const double*>(Z), lg_q1, lg2, G, r0,
                           cells, user_index, weights, dt, c, d2I, dIdw);
    } else {
        hipLaunchKernelGGL(spec_power_kernel, dim3((unsigned)((n_f + 255) / 256), grid_y),
                           dim3(256), 0, s, Z, N, G, r0, cells, user_index, weights, dt, c, d2I,
                           dIdw);
    }
    return hipGetLastError();
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
                                 double c, double2* work0, double2* work1, double2* tables,
                                 double* d2I, double* dIdw, double* dIdO, bool* parseval_done,
                                 bool first_group, hipStream_t s)
{
    *parseval_done = false;
    int lg = 0;
    while (((int64_t)1 << lg) < N)
        ++lg;
    if (N <= (int64_t)kFftTile * kFftTile) {
        // four-step: N1 = 2^lg1 in the columns step, N2 = 2^lg2 in the rows
        // step, both <= kFftTile; each workgroup holds kFftTile values (32 KiB
        // of LDS) plus its twiddles.  Rows of kFftTile / 2 let the rows step
        // take both signals of a cell and store Q; the columns step does the
        // same while N1 <= kFftTile / 2.
        const int lg2 = lg <= kFftTileLg ? 0 : std::max(kFftTileLg - 1, lg - kFftTileLg);
        const int lg1 = lg - lg2;
        const int64_t n_sig = 2 * G;
        hipLaunchKernelGGL(spec_tables_kernel, dim3(20), dim3(256), 0, s, tables, lg);
        // kFftTile values and len/2 twiddles (40 KiB for len 1024: four workgroups per CU)
        const size_t lds_a = ((size_t)kFftTile + ((size_t)1 << lg1) / 2) * sizeof(double2);
        double2* out_a = lg2 > 0 ? work0 : work1;
        if (lg2 > 0 && lg1 < kFftTileLg) {
            const int64_t tiles_per_cell = (int64_t)1 << (lg2 - (kFftTileLg - 1 - lg1));
            const int64_t tiles = G * tiles_per_cell;
            // Parseval's per-tile sums after the row step's output in work1 (G N
            // doubles of its 4 G N)
            double* part = dIdO ? reinterpret_cast<double*>(work1) + G * N : nullptr;
            if (pairs)
                hipLaunchKernelGGL(spec_cols2_kernel<true>, dim3((unsigned)tiles),
                                   dim3(kFftThreads), lds_a, s, acc, n_t, r0, G, lg1, lg2, tables,
                                   out_a, part);
            else
                hipLaunchKernelGGL(spec_cols2_kernel<false>, dim3((unsigned)tiles),
                                   dim3(kFftThreads), lds_a, s, acc, n_t, r0, G, lg1, lg2, tables,
                                   out_a, part);
            if (part) {
                hipLaunchKernelGGL(spec_parseval_parts_kernel, dim3((unsigned)((G + 255) / 256)),
                                   dim3(256), 0, s, part, tiles_per_cell, G, r0, cells, user_index,
                                   dt, c, dIdO);
                *parseval_done = true;
            }
        } else {
            const int T = kFftTile >> lg1;
            const int64_t n_cols = n_sig << lg2;
            const unsigned blocks_a = (unsigned)((n_cols + T - 1) / T);
            if (pairs)
                hipLaunchKernelGGL(spec_cols_kernel<true>, dim3(blocks_a), dim3(kFftThreads), lds_a,
                                   s, acc, n_t, r0, n_sig, lg1, lg2, tables, out_a);
            else
                hipLaunchKernelGGL(spec_cols_kernel<false>, dim3(blocks_a), dim3(kFftThreads),
                                   lds_a, s, acc, n_t, r0, n_sig, lg1, lg2, tables, out_a);
        }
        int lg_q1 = 0;
        if (lg2 > 0) {
            const size_t lds_b = ((size_t)kFftTile + ((size_t)1 << lg2) / 2) * sizeof(double2);
            if (lg2 == 10) {
                // rows of 1024 in registers, one wavefront per row of a cell
                hipLaunchKernelGGL(spec_rows_q32_kernel, dim3((unsigned)(G << lg1)), dim3(64), 0,
                                   s, work0, G, lg1, tables, reinterpret_cast<double*>(work1));
                lg_q1 = lg1;
            } else if (lg2 < kFftTileLg) {
                const int64_t tiles = G * ((int64_t)1 << (lg1 - (kFftTileLg - 1 - lg2)));
                hipLaunchKernelGGL(spec_rows_q_kernel, dim3((unsigned)tiles), dim3(kFftThreads),
                                   lds_b, s, work0, G, lg1, lg2, tables,
                                   reinterpret_cast<double*>(work1));
                lg_q1 = lg1;
            } else {
                const int R = kFftTile >> lg2;
                const unsigned blocks_b = (unsigned)(n_sig * (((int64_t)1 << lg1) / R));
                hipLaunchKernelGGL(spec_rows_kernel, dim3(blocks_b), dim3(kFftThreads), lds_b, s,
                                   work0, n_sig, lg1, lg2, tables, work1);
            }
        }
        return launch_power(work1, lg_q1, N, G, r0, cells, user_index, weights, dt, c, d2I, dIdw,
                            first_group, s);
    }
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
    return launch_power(x, 0, N, G, r0, cells, user_index, weights, dt, c, d2I, dIdw,
                        first_group, s);
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
