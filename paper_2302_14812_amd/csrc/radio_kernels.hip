// HIP kernels of libradio for gfx950 (MI355X).
//
// The deposit evaluates, for every (particle, segment, cell) triple, the
// Lienard-Wiechert field (Eq. 1) of the segment's current state and the
// arrival times of its two end states (Eq. 2), and adds the field held
// between those arrival times to the detector slots with the integrator
// weights of Sec. 3.2 / Alg. 2.  Four kernels run per deposit:
//
// 1. kinematics_kernel (Alg. 1, velocity and acceleration lines): one thread
//    per trajectory state turns (x, u) into a record with x, beta, betadot and
//    1/gamma^2 (80 bytes; 64 for the mixed modes, with (q/c) betadot and
//    1/(2 gamma^2) in single precision),
//    laid out particle-major so that the states of one particle's run are
//    contiguous.
//
// 2. order_kernel: for every tile of kTileCells detector cells, a counting
//    sort of the particles by their light-travel time to the tile's centre at
//    the chunk's middle state.  Processing particles in that order makes the
//    arrival slots a tile's cells see advance nearly monotonically.
//
// 3. ring_choice_kernel: per tile, whether the arrivals a batch touches fit
//    the small LDS ring (slow advance, many segments per slot) or need the
//    large one (a slot crossed every segment or two); it samples batches.
//
// 4. deposit_kernel: one workgroup per (tile, range of runs), launched once
//    per ring size; tiles of the other size leave at once.  Lane
//    (cell, group) = (lane % kTileCells, lane / kTileCells): the kTileCells
//    cells of the tile each get kGroups lanes, and the lanes of one group walk
//    the same particle.  Trajectories are cut into runs of kRunL segments; a
//    batch of kGroups particles (consecutive in the tile's order) x
//    (kRunL + 1) states is staged in LDS and each lane walks its particle's
//    run against its cell.  The lane integrates the held field over its
//    current slot with the exact slot-unit overlaps of Alg. 2 and emits
//    a slot's value only when its arrivals move on; emissions go to a
//    per-cell ring of slots in LDS that slides forward as the sorted batches
//    advance, and only slots leaving the ring (or emissions that fall outside
//    it) reach the detector in HBM, through atomic adds.
//
// Slot accumulator.  The detector holds, per cell and slot, the sum over
// segments of the held E and B times the segment's overlap with the slot in
// units of dt_det (Alg. 2): the slot's time average, read out as it is.  All
// updates are additive, so the ring, its fallback and the order of the
// particles only change rounding.
#include "radio_internal.h"

#include <algorithm>

#include <atomic>
#include <climits>
#include <type_traits>
#include <utility>

namespace radio {

namespace {

// pointers into LDS keep their address space, so ring updates compile to ds_*
// instructions rather than generic (flat) ones
#define RADIO_LDS __attribute__((address_space(3)))
// likewise for device memory reached through pointers that were loaded from
// memory (the job descriptors of the persistent kernel)
#define RADIO_GLOBAL __attribute__((address_space(1)))

typedef long long v2i64 __attribute__((ext_vector_type(2)));  // a 16-byte piece

template <typename P>
__device__ __forceinline__ RADIO_GLOBAL P* gptr(P* p)
{
    return (RADIO_GLOBAL P*)p;
}

// ---------------------------------------------------------------------------
// Quantities that cancel catastrophically.  Both this library and any
// reference evaluation have to round them the same way, so they are
// evaluated one IEEE operation at a time, in a fixed order, without fused
// multiply-adds.  (The slot coordinate amplifies one ulp of the arrival time
// at t_det ~ 1e5 to ~1e-7 of a slot, and 1 - n.beta ~ 1/(2 gamma^2).)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double canon_norm2(double a, double b, double c)
{
#pragma clang fp contract(off)
    return (a * a + b * b) + c * c;
}

// time of the run's state s (s < 2^53, an integer held exactly as a double)
__device__ __forceinline__ double canon_state_time(double t_first, double s, double dt)
{
#pragma clang fp contract(off)
    return t_first + s * dt;
}

// sqrt(x) correctly rounded for x = 0 and 2^-767 <= x < inf (every distance of
// physical size), with 1/sqrt(x) to an ulp or two beside it.  A hardware
// reciprocal square root seed (about 23 bits) is refined by one coupled
// Goldschmidt step, g ~ sqrt(x) and h ~ 1/(2 sqrt(x)), and g by two residual
// corrections g += (x - g^2) h, each rounded once -- the sequence the compiler
// emits for a correctly rounded double sqrt, without its rescaling of inputs
// below 2^-767 and its special-value checks (0 is handled here; inf and NaN do
// not occur).  The reciprocal is one Newton step on 1/g from 2h; for x = 0 it
// is NaN, as d (1/R) is when d = 0.
__device__ __forceinline__ double canon_sqrt(double x, double* rinv)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    double h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    g = fma(d, h, g);
    const double q = 2.0 * h;
    *rinv = fma(q, fma(-g, q, 1.0), q);
    return x == 0.0 ? 0.0 : g;
}

__device__ __forceinline__ double canon_sqrt(double x)
{
    double unused;
    return canon_sqrt(x, &unused);
}

__device__ __forceinline__ double canon_arrival(double t, double R, double inv_c)
{
#pragma clang fp contract(off)
    return t + R * inv_c;
}

// The slot coordinate (t_det - t0) / dt_det, correctly rounded, as the one IEEE
// division that defines it, without a division per state.  With the divisor b =
// dt_det, its correctly rounded reciprocal y = RN(1/b) from the host and the
// numerator x = t_det - t0:
//   q0 = RN(x y)                         within 2.5 ulp of z = x/b
//   q1 = RN(q0 + RN(x - b q0) y)         within ulp/2 + 10 u ulp   (u = 2^-53)
//   q2 = RN(q1 + (x - b q1) y)           (x - b q1 is exact here)
// Two corrections in the manner of Markstein's theorem.  q1 + (x - b q1) y =
// z + (z - q1) e with e = b y - 1, and |z - q1| <= (1/2 + 10 u) ulp(z).  A
// quotient of two doubles is never a rounding midpoint, and x - b m for a
// midpoint m is a nonzero multiple of ulp(b) ulp(z)/2, so z lies at least
// ulp(z)/(2 B) from every midpoint, B being b's significand as an integer in
// [2^52, 2^53).  q2 is therefore RN(z) whenever |e| B (1 + 20 u) < 1: true for
// most divisors (|e| <= B 2^-106) and checked for each detector on the host
// (slot_div = 0).  For the divisors where it is not, the kernels divide.
// Valid for normal x and z away from overflow and underflow (|x| >= 2^-900),
// which physical arrival times are; a non-finite x gives NaN (a dropped segment).
__device__ __forceinline__ double canon_slot(double tau, double t0, double dt_det,
                                             double inv_dt_det, bool slot_div)
{
#pragma clang fp contract(off)
    const double x = tau - t0;
    if (slot_div)
        return x / dt_det;
    double q = x * inv_dt_det;
    double r = fma(-q, dt_det, x);
    q = fma(r, inv_dt_det, q);
    r = fma(-q, dt_det, x);
    return fma(r, inv_dt_det, q);
}

// n = d/R as d * (1/R) and w = n - beta
__device__ __forceinline__ void canon_direction(const double d[3], double rinv, const double b[3],
                                                double n[3], double w[3])
{
#pragma clang fp contract(off)
    n[0] = d[0] * rinv;
    n[1] = d[1] * rinv;
    n[2] = d[2] * rinv;
    w[0] = n[0] - b[0];
    w[1] = n[1] - b[1];
    w[2] = n[2] - b[2];
}

// kappa = 1 - n.beta evaluated as (|n - beta|^2 + 1/gamma^2)/2, equal for unit n and
// free of the cancellation 1 - n.beta suffers as beta -> 1
__device__ __forceinline__ double canon_kappa(const double w[3], double inv_g2)
{
#pragma clang fp contract(off)
    return 0.5 * (((w[0] * w[0] + w[1] * w[1]) + w[2] * w[2]) + inv_g2);
}

// beta = u / sqrt(|u|^2 + 1), 1/gamma^2 = 1/(|u|^2 + 1)   (Alg. 1)
__device__ __forceinline__ void canon_kinematics(double u0, double u1, double u2, double b[3],
                                                 double* inv_g2)
{
#pragma clang fp contract(off)
    double g = canon_norm2(u0, u1, u2) + 1.0;
    double sq = __builtin_sqrt(g);
    b[0] = u0 / sq;
    b[1] = u1 / sq;
    b[2] = u2 / sq;
    *inv_g2 = 1.0 / g;
}

// betadot = (beta_s - beta_{s-1}) / dt
__device__ __forceinline__ double canon_betadot(double b, double bp, double dt)
{
#pragma clang fp contract(off)
    return (b - bp) / dt;
}

// ---------------------------------------------------------------------------
// detector updates
// ---------------------------------------------------------------------------

// Where a lane's finished slot values go in HBM.  Double path: one atomic
// add per component.  Mixed path: a compensated single-precision pair (hi, lo)
// per component; the atomic add on hi returns the old value, so the lane knows
// the exact sum the hardware rounded (old + v) and adds that rounding error
// (two-sum) to lo.
__device__ __forceinline__ float two_sum_err(float a, float b, float s)
{
#pragma clang fp contract(off)
    const float bv = s - a;
    return (a - (s - bv)) + (b - bv);
}

__device__ __forceinline__ void global_add(RADIO_GLOBAL double* row, int j, const double a[6])
{
    RADIO_GLOBAL double* q = row + (int64_t)j * 6;
#pragma unroll
    for (int k = 0; k < 6; ++k)
        __hip_atomic_fetch_add(q + k, a[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Compensated single-precision adds into the HBM pair (hi[6], lo[6]) of slot j:
// the six returning adds to hi are issued together, so that their round trips
// overlap, then the lo words take each add's rounding error.  A zero component
// adds exactly nothing (old + 0 is exact, its error 0), so no component is
// skipped: a branch per component would put the round trips in sequence.
__device__ __forceinline__ void global_add(RADIO_GLOBAL float* row, int j, const float a[6])
{
    RADIO_GLOBAL float* q = row + (int64_t)j * 12;
    float old[6];
#pragma unroll
    for (int k = 0; k < 6; ++k)
        old[k] = __hip_atomic_fetch_add(q + k, a[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int k = 0; k < 6; ++k)
        __hip_atomic_fetch_add(q + 6 + k, two_sum_err(old[k], a[k], old[k] + a[k]),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// a compensated pair (hi, lo) into the HBM pair, the same way
__device__ __forceinline__ void global_add_pair(RADIO_GLOBAL float* row, int j, const float hi[6],
                                                const float lo[6])
{
    RADIO_GLOBAL float* q = row + (int64_t)j * 12;
    float old[6];
#pragma unroll
    for (int k = 0; k < 6; ++k)
        old[k] = __hip_atomic_fetch_add(q + k, hi[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int k = 0; k < 6; ++k)
        __hip_atomic_fetch_add(q + 6 + k, two_sum_err(old[k], hi[k], old[k] + hi[k]) + lo[k],
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// position of slot j >= 0 in a ring of R slots
template <int R>
__device__ __forceinline__ int ring_pos(int j)
{
    if constexpr ((R & (R - 1)) == 0)
        return j & (R - 1);
    else
        return (int)((unsigned)j % (unsigned)R);
}

// One cell's ring of slots in LDS, covering slots [base, base + R); slot j lives
// at position j mod R.  Emissions inside go to the ring (LDS atomic add: the
// kGroups lanes of a cell share it), anything else straight to HBM.  The ring
// holds 6 doubles per slot in every mode; the emission (double or single) is
// widened and added.  Acc is the element of the HBM accumulator: double, or
// for compensated single accumulation (Acc = float) the pair hi[6], lo[6] per
// slot, which a slot leaving the ring reaches as the double split into hi and
// lo, and a bypassing emission as itself (two-sum into the pair).
template <typename Acc, int R>
struct CellSink;

template <int R>
struct CellSink<double, R> {
    static constexpr int W = 6;  // values per ring slot
    RADIO_LDS double* ring;
    RADIO_GLOBAL double* row;
    int base;
    int n_t;
    unsigned* n_bypass;
    // The ring covers [base, base + R) with 0 <= base, so a slot in it is >= 0;
    // slots at or past n_t that it holds (n_t < R) are dropped when it moves.
    template <typename F>
    __device__ __forceinline__ void flush(int j, const F a[6]) const
    {
        double v[6];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            v[k] = (double)a[k];
        if ((unsigned)(j - base) < (unsigned)R) {
            RADIO_LDS double* q = ring + ring_pos<R>(j) * W;
#pragma unroll
            for (int k = 0; k < 6; ++k)
                __hip_atomic_fetch_add(q + k, v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else if ((unsigned)j < (unsigned)n_t) {
            *n_bypass += 1u;
            global_add(row, j, v);
        }
    }
};

template <int R>
struct CellSink<float, R> {
    static constexpr int W = 6;  // ring values per slot
    RADIO_LDS double* ring;
    RADIO_GLOBAL float* row;      // hi[6], lo[6] per slot
    int base;
    int n_t;
    unsigned* n_bypass;
    __device__ __forceinline__ void flush(int j, const float a[6]) const
    {
        if ((unsigned)(j - base) < (unsigned)R) {
            RADIO_LDS double* q = ring + ring_pos<R>(j) * W;
#pragma unroll
            for (int k = 0; k < 6; ++k)
                __hip_atomic_fetch_add(q + k, (double)a[k], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        } else if ((unsigned)j < (unsigned)n_t) {
            *n_bypass += 1u;
            global_add(row, j, a);
        }
    }
};

// ---------------------------------------------------------------------------
// the lane's open slot
// ---------------------------------------------------------------------------

// For the run being processed the lane integrates the held field over its
// current slot J (V); when the run leaves slot J, V is final and is emitted.
// Every overlap is the exact slot-unit overlap of the integrator definition
// (Alg. 2), so each segment contributes the same numbers the definition
// gives; only the order of the additions differs.  Slots outside [0, n_t)
// are dropped by the sink, which is how the window clips (Alg. 1).
//
// The carry keeps J + 1 as a double (J1) and the bound `lim` of the fast path:
// a segment [a, b] with a <= b < lim starts in the open slot (a in [J, J+1)),
// with J >= 0, and ends below n_t, so it lies inside the window.  lim is n_t
// while the next segment's start is known to lie in the open slot, inside the
// window, and -inf otherwise; such a segment takes the general path, which
// also counts the segments that reach outside [0, n_t] (clipped) and those
// that run backward.

template <typename T>
struct Carry {
    double J1;   // open slot + 1; the slot may lie outside [0, n_t), far below 0 when none is open
    double lim;  // fast-path bound of the next segment
    T V[6];      // integral of the held field over the open slot so far
};

template <typename T>
__device__ __forceinline__ void carry_open(Carry<T>& C, double J)
{
    C.J1 = J + 1.0;
#pragma unroll
    for (int k = 0; k < 6; ++k)
        C.V[k] = T(0);
}

// the fast-path bound when the open slot is J and the next segment starts at a
__device__ __forceinline__ double fast_limit(double J, double a, double ntd)
{
    return ((J >= 0.0) & (a >= J) & (a < J + 1.0)) ? ntd : -INFINITY;
}

// a segment between a and b reaches outside the window [0, n_t] (a NaN end is
// not counted as outside)
__device__ __forceinline__ unsigned clipped(double a, double b, double ntd)
{
    return ((a < 0.0) | (b < 0.0) | (a > ntd) | (b > ntd)) ? 1u : 0u;
}

// The ends of the segment between a and b, ordered and clamped to [0, n_t].
// Compares and selects only: min/max instructions would make the compiler
// quiet the operands of every state, general path taken or not.  A NaN end
// gives a NaN bound, which the callers' lo < hi test treats as empty.
__device__ __forceinline__ void clamp_segment(double a, double b, double ntd, double& lo,
                                              double& hi)
{
    const bool back = b < a;
    const double mn = back ? b : a, mx = back ? a : b;
    lo = mn < 0.0 ? 0.0 : (mn > ntd ? ntd : mn);
    hi = mx < 0.0 ? 0.0 : (mx > ntd ? ntd : mx);
}

// General case: hold F over the slot-coordinate interval between a and b,
// clipped to [0, n_t]; any order, any length.  A segment that does not start
// in the open slot closes it first, which is exact because deposits add.
// Backward segments are counted here (the fast path takes none).
template <typename T, typename Sink>
__device__ __forceinline__ void add_segment_general(Carry<T>& C, const Sink& sink, int n_t,
                                                    double a, double b, const T F[6],
                                                    unsigned& n_back, unsigned& n_clip)
{
    const double ntd = (double)n_t;
    n_back += (b < a) ? 1u : 0u;
    n_clip += clipped(a, b, ntd);
    double lo, hi;
    clamp_segment(a, b, ntd, lo, hi);
    if (lo < hi) {  // else empty, entirely outside, or NaN
        const double fl = floor(lo);  // < n_t
        const double fh = floor(hi);  // <= n_t; n_t only when hi reaches the end
        if (fl != C.J1 - 1.0) {
            sink.flush((int)(C.J1 - 1.0), C.V);
            carry_open(C, fl);
        }
        if (fh == fl) {
            const T w = T(hi - lo);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                C.V[k] += F[k] * w;
        } else {
            const T wa = T((fl + 1.0) - lo);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                C.V[k] += F[k] * wa;
            const int jl = (int)fl, jh = (int)fh;
            sink.flush(jl, C.V);
            for (int j = jl + 1; j < jh; ++j)  // whole slots hold F
                sink.flush(j, F);
            const T wb = T(hi - fh);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                C.V[k] = F[k] * wb;
            C.J1 = fh + 1.0;
        }
    }
    C.lim = fast_limit(C.J1 - 1.0, b, ntd);
}

// One segment [a, b] of a lane's run.  Fast path (a <= b < lim): the overlaps
// are b - a (same slot) or J + 1 - a, whole slots, and b - floor(b) -- those
// of the definition -- and the emissions are guarded by the crossing count
// only.  Everything else goes through add_segment_general.
template <typename T, typename Sink>
__device__ __forceinline__ void add_segment(Carry<T>& C, const Sink& sink, int n_t, double a,
                                            double b, const T F[6], unsigned& n_back,
                                            unsigned& n_clip)
{
    if ((b >= a) & (b < C.lim)) {
        const bool leaves = b >= C.J1;  // the segment leaves the open slot
        const T w0 = T((leaves ? C.J1 : b) - a);
#pragma unroll
        for (int k = 0; k < 6; ++k)
            C.V[k] += F[k] * w0;
        if (leaves) {
            const double fb = floor(b);
            sink.flush((int)C.J1 - 1, C.V);
            if (fb > C.J1)  // whole slots J + 1 .. floor(b) - 1 hold F
                for (int j = (int)C.J1; j < (int)fb; ++j)
                    sink.flush(j, F);
            const T wb = T(b - fb);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                C.V[k] = F[k] * wb;
            C.J1 = fb + 1.0;
        }
    } else {
        add_segment_general(C, sink, n_t, a, b, F, n_back, n_clip);
    }
}

// The linear rule: the field runs from Fa at slot coordinate a to Fb at b, and
// each slot receives its overlap with the segment times the interpolant at the
// overlap's midpoint (the exact integral of a linear function).  Same fast and
// general paths as add_segment.
template <typename T>
__device__ __forceinline__ void lerp_field(const T Fa[6], const T dF[6], T f, T out[6])
{
#pragma unroll
    for (int k = 0; k < 6; ++k)
        out[k] = Fa[k] + dF[k] * f;
}

template <typename T, typename Sink>
__device__ __forceinline__ void add_segment_linear_general(Carry<T>& C, const Sink& sink, int n_t,
                                                           double a, double b, const T Fa[6],
                                                           const T dF[6], double inv_len,
                                                           unsigned& n_back, unsigned& n_clip)
{
    const double ntd = (double)n_t;
    n_back += (b < a) ? 1u : 0u;
    n_clip += clipped(a, b, ntd);
    double lo, hi;
    clamp_segment(a, b, ntd, lo, hi);
    if (lo < hi) {
        const double fl = floor(lo);
        const double fh = floor(hi);
        if (fl != C.J1 - 1.0) {
            sink.flush((int)(C.J1 - 1.0), C.V);
            carry_open(C, fl);
        }
        T F[6];
        auto piece = [&](double p, double q) {  // the interpolant times the overlap [p, q]
            lerp_field(Fa, dF, T(0.5 * ((p - a) + (q - a)) * inv_len), F);
            const T w = T(q - p);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                F[k] *= w;
        };
        if (fh == fl) {
            piece(lo, hi);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                C.V[k] += F[k];
        } else {
            const int jl = (int)fl, jh = (int)fh;
            piece(lo, fl + 1.0);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                C.V[k] += F[k];
            sink.flush(jl, C.V);
            for (int j = jl + 1; j < jh; ++j) {
                piece((double)j, (double)(j + 1));
                sink.flush(j, F);
            }
            piece(fh, hi);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                C.V[k] = F[k];
            C.J1 = fh + 1.0;
        }
    }
    C.lim = fast_limit(C.J1 - 1.0, b, ntd);
}

template <typename T, typename Sink>
__device__ __forceinline__ void add_segment_linear(Carry<T>& C, const Sink& sink, int n_t,
                                                   double a, double b, const T Fa[6],
                                                   const T Fb[6], unsigned& n_back,
                                                   unsigned& n_clip)
{
    if (a == b) {  // no length: nothing to hold, and the carry still fits the next start
        n_clip += clipped(a, b, (double)n_t);
        return;
    }
    T dF[6];
#pragma unroll
    for (int k = 0; k < 6; ++k)
        dF[k] = Fb[k] - Fa[k];
    const double inv_len = 1.0 / (b - a);
    if ((b > a) & (b < C.lim)) {
        const double Jd = C.J1 - 1.0;
        const double e0 = b < C.J1 ? b : C.J1;
        T F[6];
        lerp_field(Fa, dF, T(0.5 * (e0 - a) * inv_len), F);
        const T w0 = T(e0 - a);
#pragma unroll
        for (int k = 0; k < 6; ++k)
            C.V[k] += F[k] * w0;
        if (b >= C.J1) {
            const double fb = floor(b);
            const int J = (int)C.J1 - 1;
            const int n = (int)(fb - C.J1) + 1;  // slots crossed
            sink.flush(J, C.V);
            for (int i = 1; i < n; ++i) {  // whole slots: the interpolant at their middle
                lerp_field(Fa, dF, T(0.5 * ((Jd + (double)i - a) + (Jd + (double)(i + 1) - a)) *
                                     inv_len),
                           F);
                sink.flush(J + i, F);
            }
            lerp_field(Fa, dF, T(0.5 * ((fb - a) + (b - a)) * inv_len), F);
            const T wb = T(b - fb);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                C.V[k] = F[k] * wb;
            C.J1 = fb + 1.0;
        }
    } else {
        add_segment_linear_general(C, sink, n_t, a, b, Fa, dF, inv_len, n_back, n_clip);
    }
}

// ---------------------------------------------------------------------------
// field evaluation
// ---------------------------------------------------------------------------

struct Consts {
    double t0, inv_dt_det, inv_c;
    double kR;      // inv_c * inv_dt_det: slots per unit of distance (mixed modes)
    double dt_det;  // the slot width (the divisor of the double slot coordinate)
    bool slot_div;  // the double slot coordinate takes a division (see canon_slot)
};

__device__ __forceinline__ double canon_slot(double tau, const Consts& K)
{
    return canon_slot(tau, K.t0, K.dt_det, K.inv_dt_det, K.slot_div);
}

// E and B of Eq. 1 from the unit vector n to the cell, w = n - beta, 1/kappa,
// 1/R and the state's 1/gamma^2 and betadot, for a charge with qc = q/c and
// qv = q times the weight of the velocity term.  The acceleration term is
// regrouped with the identity n x (w x bd) = w (n.bd) - bd (n.w):
//   E = c1 w - c2 bd,  c1 = (qc n.bd + qv g2i / R) / (kappa^3 R),
//                      c2 = qc (n.w) / (kappa^3 R),
//   B = n x E.
// nwk is (n.w)/kappa.  For a unit n, n.w = 1 - n.beta = kappa and nwk = 1,
// which the single-precision field (lw_fields_mixed) takes: it is the more
// accurate value there.  The double field passes the product of its rounded n
// and w, as the cross products of Eq. 1 would use them (with kappa of order
// 1/gamma^2, the last bits of |n| shift n.w by up to ~1e-12 of itself).
template <typename T>
__device__ __forceinline__ void lw_fields(const T n[3], const T w[3], T kinv, T rinv, T g2i,
                                          const T bd[3], T qc, T qv, T nwk, T F[6])
{
    const T nbd = n[0] * bd[0] + n[1] * bd[1] + n[2] * bd[2];
    const T rk2 = rinv * (kinv * kinv);
    const T c1 = (qc * nbd + qv * g2i * rinv) * (rk2 * kinv);
    const T c2 = qc * rk2 * nwk;
    const T E0 = c1 * w[0] - c2 * bd[0];
    const T E1 = c1 * w[1] - c2 * bd[1];
    const T E2 = c1 * w[2] - c2 * bd[2];
    F[0] = E0;
    F[1] = E1;
    F[2] = E2;
    F[3] = n[1] * E2 - n[2] * E1;
    F[4] = n[2] * E0 - n[0] * E2;
    F[5] = n[0] * E1 - n[1] * E0;
}

// 1/x from the hardware reciprocal refined by two Newton steps (within an ulp
// or two; used where Eq. 1 needs no particular rounding)
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Lienard-Wiechert E, B (Eq. 1) at a cell from one staged state, all in double;
// returns the state's slot coordinate.  Only the arrival time (R and tau) is
// rounded canonically; n, w, kappa and the field, which decide no slot, use
// FMAs, 1/R from canon_sqrt and a Newton reciprocal for 1/kappa (within an ulp
// or two of the correctly rounded values).
__device__ __forceinline__ double field_fp64(const double xc[3], const RecF64& st, double t_s,
                                             double qc, double qv, const Consts& K, double F[6])
{
    double d[3] = {xc[0] - st.x[0], xc[1] - st.x[1], xc[2] - st.x[2]};
    double rinv;
    const double R = canon_sqrt(canon_norm2(d[0], d[1], d[2]), &rinv);
    double tau = canon_arrival(t_s, R, K.inv_c);
    const double n[3] = {d[0] * rinv, d[1] * rinv, d[2] * rinv};
    const double w[3] = {n[0] - st.b[0], n[1] - st.b[1], n[2] - st.b[2]};
    // kappa = (|n - beta|^2 + 1/gamma^2) / 2, as canon_kappa but fused
    const double kinv =
        recip(0.5 * fma(w[0], w[0], fma(w[1], w[1], fma(w[2], w[2], st.g2i))));
    const double nwk = (n[0] * w[0] + n[1] * w[1] + n[2] * w[2]) * kinv;
    lw_fields<double>(n, w, kinv, rinv, st.g2i, st.bd, qc, qv, nwk, F);
    return canon_slot(tau, K);
}

// R = |d| and 1/R from one hardware reciprocal square root (about 23 correct
// bits) refined by a Newton step for 1/R and a residual correction for R,
// both to ~1e-15 relative -- enough for arrival times of 1e5 against slots of
// 1e-4 -- at a third of the cost of a correctly rounded sqrt plus a divide.
__device__ __forceinline__ void fast_norm(double R2, double* R, double* rinv)
{
    double y = __builtin_amdgcn_rsq(R2);
    y = y * fma(-0.5 * R2 * y, y, 1.5);
    double g = R2 * y;
    double r = fma(-g, g, R2);
    *R = fma(r, 0.5 * y, g);
    *rinv = y;
}

// |d|^2 for fast_norm, plus the smallest normal double.  That changes nothing
// for distances above ~1e-146, and a state exactly at a cell (d = 0) then gets
// R ~ 1e-154 and a finite slot coordinate -- the canonical R = 0 moves the
// slot coordinate by no more -- instead of 0 * inf.  Its field is not finite,
// as the definition's is there.
__device__ __forceinline__ double norm2_fast(double d0, double d1, double d2)
{
    return fma(d2, d2, fma(d1, d1, fma(d0, d0, 0x1p-1022)));
}

// lw_fields in single precision for a mixed-precision record, whose betadot
// already carries the factor q/c (bdq = q bd / c) and whose g2ih is 1/(2 gamma^2):
// kappa = |w|^2 / 2 + g2ih, and with n.w = kappa for a unit n,
//   E = c1 w - bdq / (kappa^2 R),  c1 = (n.bdq + qvg / R) / (kappa^3 R),
// where qvg = qv g2i = 2 qv g2ih.
__device__ __forceinline__ void lw_fields_mixed(const float n[3], const float w[3], float rinv,
                                                const RecMix& st, float qv2, float F[6])
{
    const float kinv =
        __builtin_amdgcn_rcpf(fmaf(0.5f, w[0] * w[0] + w[1] * w[1] + w[2] * w[2], st.g2ih));
    const float nbd = n[0] * st.bdq[0] + n[1] * st.bdq[1] + n[2] * st.bdq[2];
    const float rk2 = rinv * (kinv * kinv);
    const float c1 = fmaf(qv2 * st.g2ih, rinv, nbd) * (rk2 * kinv);
    const float E0 = c1 * w[0] - rk2 * st.bdq[0];
    const float E1 = c1 * w[1] - rk2 * st.bdq[1];
    const float E2 = c1 * w[2] - rk2 * st.bdq[2];
    F[0] = E0;
    F[1] = E1;
    F[2] = E2;
    F[3] = n[1] * E2 - n[2] * E1;
    F[4] = n[2] * E0 - n[0] * E2;
    F[5] = n[0] * E1 - n[1] * E0;
}

// The mixed-precision field: double for what cancels (arrival time, slot
// coordinate, n - beta), single for the rest of Eq. 1, kappa included (a sum
// of positive terms formed from the double difference n - beta).  ub is the
// state's (t_s - t0) / dt_det; the slot coordinate is ub + R / (c dt_det).
// qv2 = 2 q times the weight of the velocity term.
__device__ __forceinline__ double field_mixed(const double xc[3], const RecMix& st, double ub,
                                              float qv2, const Consts& K, float F[6])
{
    double d[3] = {xc[0] - st.x[0], xc[1] - st.x[1], xc[2] - st.x[2]};
    double R, rinv;
    fast_norm(norm2_fast(d[0], d[1], d[2]), &R, &rinv);
    const double u = fma(R, K.kR, ub);
    double nd[3] = {d[0] * rinv, d[1] * rinv, d[2] * rinv};
    double wd[3] = {nd[0] - st.b[0], nd[1] - st.b[1], nd[2] - st.b[2]};
    const float n[3] = {(float)nd[0], (float)nd[1], (float)nd[2]};
    const float w[3] = {(float)wd[0], (float)wd[1], (float)wd[2]};
    lw_fields_mixed(n, w, (float)rinv, st, qv2, F);
    return u;
}

// Far-field geometry (Eq. 3): the cell's direction and distance from the
// origin, fc = {n0, n1, n2, R_cell}; arrival t + (R_cell - x.n) (1/c), the
// dot product in a fixed order without FMA.
__device__ __forceinline__ double canon_far_arrival(double t, const double fc[4],
                                                    const double x[3], double inv_c)
{
#pragma clang fp contract(off)
    const double dot = (x[0] * fc[0] + x[1] * fc[1]) + x[2] * fc[2];
    return t + (fc[3] - dot) * inv_c;
}

// w = n - beta with the cell's direction
__device__ __forceinline__ void canon_far_w(const double fc[4], const double b[3], double w[3])
{
#pragma clang fp contract(off)
    w[0] = fc[0] - b[0];
    w[1] = fc[1] - b[1];
    w[2] = fc[2] - b[2];
}

// ub = (t_s - t0) / dt_det, as for field_mixed
__device__ __forceinline__ double slot_far_mixed(const double fc[4], const double x[3], double ub,
                                                 const Consts& K)
{
    return fma(fc[3] - (x[0] * fc[0] + x[1] * fc[1] + x[2] * fc[2]), K.kR, ub);
}

__device__ __forceinline__ double slot_far_fp64(const double fc[4], const double x[3], double t_s,
                                                const Consts& K)
{
    return canon_slot(canon_far_arrival(t_s, fc, x, K.inv_c), K);
}

// Eq. 1 with the far-field geometry n = n_cell, R = R_cell; Rinv = 1/R_cell
__device__ __forceinline__ double field_far_fp64(const double fc[4], double Rinv,
                                                 const RecF64& st, double t_s, double qc,
                                                 double qv, const Consts& K, double F[6])
{
    double w[3];
    canon_far_w(fc, st.b, w);
    const double kinv = recip(canon_kappa(w, st.g2i));
    const double nwk = (fc[0] * w[0] + fc[1] * w[1] + fc[2] * w[2]) * kinv;
    lw_fields<double>(fc, w, kinv, Rinv, st.g2i, st.bd, qc, qv, nwk, F);
    return slot_far_fp64(fc, st.x, t_s, K);
}

__device__ __forceinline__ double field_far_mixed(const double fc[4], double Rinv,
                                                  const RecMix& st, double ub, float qv2,
                                                  const Consts& K, float F[6])
{
    const double u = slot_far_mixed(fc, st.x, ub, K);
    const double wd[3] = {fc[0] - st.b[0], fc[1] - st.b[1], fc[2] - st.b[2]};
    const float n[3] = {(float)fc[0], (float)fc[1], (float)fc[2]};
    const float w[3] = {(float)wd[0], (float)wd[1], (float)wd[2]};
    lw_fields_mixed(n, w, (float)Rinv, st, qv2, F);
    return u;
}

// 1/gamma^2 of a staged state
__device__ __forceinline__ double rec_g2i(const RecF64& st) { return st.g2i; }
__device__ __forceinline__ double rec_g2i(const RecMix& st) { return 2.0 * (double)st.g2ih; }

// Lienard-Wiechert potentials phi = q/(kappa R), A = q beta/(kappa R) at a
// staged state (the potentials option): F = (A_x, A_y, A_z, phi, 0, 0).  FAR:
// the cell's direction and distance.  (The caller takes the slot coordinate
// from the same expression its other deposits use.)
template <bool FAR, typename Rec, typename T>
__device__ __forceinline__ void potentials_at(const double xc[3], const double fc[4],
                                              const Rec& st, double q, T F[6])
{
    double kap, rinv;
    if constexpr (FAR) {
        double w[3];
        canon_far_w(fc, st.b, w);
        kap = canon_kappa(w, rec_g2i(st));
        rinv = 1.0 / fc[3];
    } else {
        double d[3] = {xc[0] - st.x[0], xc[1] - st.x[1], xc[2] - st.x[2]};
        const double R = canon_sqrt(canon_norm2(d[0], d[1], d[2]));
        rinv = 1.0 / R;
        double n[3], w[3];
        canon_direction(d, rinv, st.b, n, w);
        kap = canon_kappa(w, rec_g2i(st));
    }
    const double phi = q * rinv / kap;
    F[0] = T(phi * st.b[0]);
    F[1] = T(phi * st.b[1]);
    F[2] = T(phi * st.b[2]);
    F[3] = T(phi);
    F[4] = T(0);
    F[5] = T(0);
}

__device__ __forceinline__ double slot_coord_fp64(const double xc[3], const double x[3],
                                                  double t_s, const Consts& K)
{
    double d[3] = {xc[0] - x[0], xc[1] - x[1], xc[2] - x[2]};
    const double R = canon_sqrt(canon_norm2(d[0], d[1], d[2]));
    return canon_slot(canon_arrival(t_s, R, K.inv_c), K);
}

// ub = (t_s - t0) / dt_det, as for field_mixed
__device__ __forceinline__ double slot_coord_mixed(const double xc[3], const double x[3],
                                                   double ub, const Consts& K)
{
    double d[3] = {xc[0] - x[0], xc[1] - x[1], xc[2] - x[2]};
    double R, rinv;
    fast_norm(norm2_fast(d[0], d[1], d[2]), &R, &rinv);
    return fma(R, K.kR, ub);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// One thread per (particle, state): the state record of mode M, particle-major.
// betadot of a state: kBdBackward (beta_s - beta_{s-1})/dt, zero at the chunk's first
// state (it carries no segment); kBdBackwardFirst the same but the forward difference
// at the first state (its field is held by the previous-state rule); kBdCentred
// (beta_{s+1} - beta_{s-1})/(2 dt), one-sided at the chunk's ends (linear rule)
constexpr int kBdBackward = 0, kBdBackwardFirst = 1, kBdCentred = 2;

// Mixed-precision records carry the particle's q/c in betadot and half of
// 1/gamma^2, the forms their field takes (q: [n_p] or nullptr, all -1).  x and
// u point at the job's state 0, with components `stride` elements apart; they
// hold states s_lo <= 0 .. s_hi >= n_s (a time slice of a longer chunk reads
// its neighbours, so that its records equal those of the whole chunk).
template <int M>
__global__ __launch_bounds__(256) void kinematics_kernel(const double* __restrict__ x,
                                                         const double* __restrict__ u,
                                                         const double* __restrict__ q,
                                                         int64_t n_p, int64_t n_s, int64_t stride,
                                                         int64_t s_lo, int64_t s_hi, double dt,
                                                         double inv_c, int bd_rule,
                                                         void* __restrict__ recs_out)
{
    using Rec = typename std::conditional<M == kModeF64, RecF64, RecMix>::type;
    Rec* recs = reinterpret_cast<Rec*>(recs_out);
    const int64_t n_states = n_s + 1;
    const int64_t total = n_p * n_states;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / n_p;  // consecutive threads read consecutive particles
        const int64_t p = i - s * n_p;
        const int64_t off = s * n_p + p;
        Rec r;
        r.x[0] = x[off];
        r.x[1] = x[off + stride];
        r.x[2] = x[off + 2 * stride];
        double g2i;
        canon_kinematics(u[off], u[off + stride], u[off + 2 * stride], r.b, &g2i);
        double bd[3] = {0.0, 0.0, 0.0};
        if (bd_rule == kBdCentred && s_hi > s_lo) {
            const int64_t sa = s > s_lo ? s - 1 : s_lo;
            const int64_t sb = s < s_hi ? s + 1 : s_hi;
            double ba[3], bb[3], g;
            const int64_t oa = sa * n_p + p, ob = sb * n_p + p;
            canon_kinematics(u[oa], u[oa + stride], u[oa + 2 * stride], ba, &g);
            canon_kinematics(u[ob], u[ob + stride], u[ob + 2 * stride], bb, &g);
#pragma unroll
            for (int c = 0; c < 3; ++c)
                bd[c] = canon_betadot(bb[c], ba[c], (double)(sb - sa) * dt);
        } else if (s > s_lo || (bd_rule == kBdBackwardFirst && s_hi > s_lo)) {
            // backward difference; at the first state, the forward one
            double bo[3], go;
            const int64_t o2 = s > s_lo ? off - n_p : off + n_p;
            canon_kinematics(u[o2], u[o2 + stride], u[o2 + 2 * stride], bo, &go);
#pragma unroll
            for (int c = 0; c < 3; ++c)
                bd[c] = s > s_lo ? canon_betadot(r.b[c], bo[c], dt)
                                 : canon_betadot(bo[c], r.b[c], dt);
        }
        if constexpr (M == kModeF64) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
                r.bd[c] = bd[c];
            r.g2i = g2i;
        } else {
            const double qc = (q ? q[p] : -1.0) * inv_c;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                r.bdq[c] = (float)(qc * bd[c]);
            r.g2ih = (float)(0.5 * g2i);
        }
        recs[p * n_states + s] = r;
    }
}

// Counting sort of the particles of one chunk, per tile, by the light-travel
// distance from the tile's centre to each particle at state s_key, in bins of
// one slot (widened if the spread needs more than kOrderBins).  perm[tile][i]
// is the i-th particle in that order.
constexpr int kOrderBins = 4096;

__global__ __launch_bounds__(256) void order_kernel(const double* __restrict__ x, int64_t n_p,
                                                    int64_t n_s, int64_t xs_stride,
                                                    int64_t n_tiles, int64_t tile_cells,
                                                    int64_t steps_per_group,
                                                    const double* __restrict__ cells, int64_t n_c,
                                                    double inv_c, double inv_dt_det,
                                                    int32_t* __restrict__ perm)
{
    __shared__ unsigned hist[kOrderBins];
    __shared__ double red_lo[256], red_hi[256];
    __shared__ double ctr[3];
    const int tid = threadIdx.x;
    const int64_t tile = blockIdx.x % n_tiles;
    const int64_t group = blockIdx.x / n_tiles;
    // the group's middle state
    const int64_t s_key = min(n_s, group * steps_per_group + steps_per_group / 2);
    const int64_t c0 = tile * tile_cells;
    const int64_t c1 = min(c0 + tile_cells, n_c);
    if (tid < 3) {
        double s = 0.0;
        for (int64_t c = c0; c < c1; ++c)
            s += cells[3 * c + tid];
        ctr[tid] = s / (double)(c1 - c0);
    }
    for (int i = tid; i < kOrderBins; i += 256)
        hist[i] = 0u;
    __syncthreads();
    const int64_t stride = xs_stride;
    const int64_t base = s_key * n_p;
    const double cx = ctr[0], cy = ctr[1], cz = ctr[2];
    auto key = [&](int64_t p) {
        const double d0 = cx - x[base + p];
        const double d1 = cy - x[base + p + stride];
        const double d2 = cz - x[base + p + 2 * stride];
        return __builtin_sqrt(d0 * d0 + d1 * d1 + d2 * d2) * (inv_c * inv_dt_det);
    };
    double lo = 1e300, hi = -1e300;
    for (int64_t p = tid; p < n_p; p += 256) {
        const double k = key(p);
        if (k == k) {
            lo = fmin(lo, k);
            hi = fmax(hi, k);
        }
    }
    red_lo[tid] = lo;
    red_hi[tid] = hi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            red_lo[tid] = fmin(red_lo[tid], red_lo[tid + s]);
            red_hi[tid] = fmax(red_hi[tid], red_hi[tid + s]);
        }
        __syncthreads();
    }
    lo = red_lo[0];
    hi = red_hi[0];
    const double span = hi > lo ? hi - lo : 0.0;
    const double width = span < (double)(kOrderBins - 1) ? 1.0 : span / (double)(kOrderBins - 1);
    auto bin_of = [&](int64_t p) {
        const double k = key(p);
        double b = (k - lo) / width;
        b = (b == b) ? fmin(fmax(b, 0.0), (double)(kOrderBins - 1)) : (double)(kOrderBins - 1);
        return (int)b;
    };
    for (int64_t p = tid; p < n_p; p += 256)
        atomicAdd(&hist[bin_of(p)], 1u);
    __syncthreads();
    if (tid == 0) {  // exclusive scan (4096 entries, once per tile)
        unsigned run = 0;
        for (int i = 0; i < kOrderBins; ++i) {
            const unsigned h = hist[i];
            hist[i] = run;
            run += h;
        }
    }
    __syncthreads();
    int32_t* out = perm + (group * n_tiles + tile) * n_p;
    for (int64_t p = tid; p < n_p; p += 256) {
        const unsigned pos = atomicAdd(&hist[bin_of(p)], 1u);
        out[pos] = (int32_t)p;
    }
}

// For every tile, whether its batches take the large slot ring.  The small
// ring keeps four workgroups on a CU, the large one two, so the large ring
// pays only where the small one would send many emissions to HBM.  The
// kernel replays sampled batches (the first and the middle run, at eight
// places of the tile's particle order) at the tile's first cell: it places
// a small ring the way the deposit does (below the batch's earliest start)
// and counts the slots a lane would emit outside it.  Above kRingBypassLimit
// such emissions per interaction the tile takes the large ring.  Only speed
// depends on this choice: emissions outside a ring go to HBM directly.
constexpr double kRingBypassLimit = 0.05;   // emissions to HBM per interaction

__global__ __launch_bounds__(256) void ring_choice_kernel(const char* __restrict__ recs,
                                                          int64_t rec_size,
                                                          const int32_t* __restrict__ perm,
                                                          int64_t n_tiles, int64_t runs_per_group,
                                                          const double* __restrict__ cells,
                                                          const double* __restrict__ far,
                                                          int64_t n_c, int64_t n_p, int64_t n_s,
                                                          int64_t n_runs, double t_first,
                                                          int64_t s0, double dt, double t0,
                                                          double inv_dt_det, double inv_c,
                                                          int64_t n_t, int tile_cells, int groups,
                                                          int run_l, uint8_t* __restrict__ sel)
{
    // one thread per sampled particle: 256 / groups sampled batches, half of them
    // in the first run and half in the middle one
    const int n_samples = 256 / groups;
    const int kChoiceBatches = n_samples / 2;
    __shared__ int start[64];
    __shared__ unsigned out_count, segs;
    const int tid = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int64_t c0 = tile * tile_cells;
    if (tid < n_samples)
        start[tid] = INT_MAX;
    if (tid == 0) {
        out_count = 0u;
        segs = 0u;
    }
    const int smp = tid / groups;  // sampled batch
    const int gg = tid % groups;   // particle within it
    const int64_t n_states = n_s + 1;
    const int64_t n_batches = (n_p + groups - 1) / groups;
    const int64_t run = (smp < kChoiceBatches) ? 0 : n_runs / 2;
    const int64_t bt = (2 * (int64_t)(smp % kChoiceBatches) + 1) * n_batches / (2 * kChoiceBatches);
    const int64_t pi = bt * groups + gg;
    const int64_t s_a = run * run_l;
    const int len = (int)min((int64_t)run_l, n_s - s_a);
    const bool on = smp < n_samples && pi < n_p && len > 0;
    const double* xc = cells + 3 * c0;
    const double* fc = far ? far + 4 * c0 : nullptr;
    const int32_t* order = perm + ((run / runs_per_group) * n_tiles + tile) * n_p;  // once a thread
    const char* pr = on ? recs + ((int64_t)order[pi] * n_states + s_a) * rec_size : nullptr;
    // position of state k of this lane's particle: the first three doubles of its record
    auto pos = [&](int k) { return reinterpret_cast<const double*>(pr + (int64_t)k * rec_size); };
    auto slot_of = [&](const double* x, int64_t st) {
        double dist;
        if (fc) {
            dist = fc[3] - (x[0] * fc[0] + x[1] * fc[1] + x[2] * fc[2]);
        } else {
            const double d0 = xc[0] - x[0], d1 = xc[1] - x[1], d2 = xc[2] - x[2];
            dist = __builtin_sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        }
        const double u = ((t_first + (double)(s0 + st) * dt) + dist * inv_c - t0) * inv_dt_det;
        return (u == u) ? fmin(fmax(u, -2.0), (double)n_t + 2.0) : -2.0;
    };
    __syncthreads();
    if (on)
        atomicMin(&start[smp], (int)floor(slot_of(pos(0), s_a)));
    __syncthreads();
    if (on) {
        // the small ring of this batch, placed as the deposit places it
        const int base = (int)fmin(fmax((double)start[smp] - (double)kRingMargin, 0.0),
                                   fmax((double)(n_t - kRingSmall), 0.0));
        unsigned outside = 0u;
        auto emit = [&](int j) {
            if (j >= 0 && j < n_t && (j < base || j >= base + kRingSmall))
                ++outside;
        };
        int J = (int)floor(slot_of(pos(0), s_a));
        for (int k = 1; k <= len; ++k) {
            const int jk = (int)floor(slot_of(pos(k), s_a + k));
            for (int j = min(J, jk); j < max(J, jk); ++j)  // slots the lane leaves
                emit(j);
            J = jk;
        }
        emit(J);  // the run's last slot
        atomicAdd(&out_count, outside);
        atomicAdd(&segs, (unsigned)len);
    }
    __syncthreads();
    if (tid == 0)
        sel[tile] = (segs > 0u && (double)out_count > kRingBypassLimit * (double)segs) ? 1 : 0;
}

// M: arithmetic of the deposit (field in double or single; accumulation in
// double or compensated single pairs)
template <int M>
struct ModeTypes {
    static constexpr bool MIX = (M != kModeF64);
    using T = typename std::conditional<MIX, float, double>::type;  // field and lane carry
    using Acc = typename std::conditional<M == kModeMixTwoSum, float, double>::type;
    using Rec = typename std::conditional<MIX, RecMix, RecF64>::type;  // staged state record
};

// Segments a workgroup of shape SH stages per batch: a whole run with the small
// ring; with the large ring at most kLargeStage (a run of more is staged in
// parts), because the arrivals of a batch must fit the ring's span.
template <int R, int SH>
constexpr int kSubRun =
    (R == kRingLarge && shape_run(SH) > kLargeStage) ? kLargeStage : shape_run(SH);

// LDS of one deposit workgroup of shape SH with rings of R slots
template <int M, int R, int SH>
struct DepositShared {
    using Acc = typename ModeTypes<M>::Acc;
    static constexpr int TC = shape_cells(SH);   // cells per tile
    static constexpr int GR = shape_groups(SH);  // particles per batch
    // one cell's ring, padded by one word so that the rings of the tile's
    // cells, which one instruction updates together, start in different banks
    static constexpr int kStride = R * CellSink<Acc, R>::W + 1;
    static constexpr int L = kSubRun<R, SH>;
    static_assert(shape_run(SH) % L == 0, "a run is a whole number of staged parts");
    typename ModeTypes<M>::Rec rec[GR][L + 1];  // staged batch: L segments per group
    double sq[GR];                      // its charges
    double tk[L + 1];                   // its states' time arguments (the same for every lane)
    double ring[TC * kStride];          // per-cell slot rings
    int nb[2][TC];                      // per cell: lowest start slot of a coming batch
    int ord[2][GR];                     // particles of the staged rows, per batch parity
    unsigned long long cnt[kCounters];  // clipped, nonmonotone, bypassed, large-ring interactions
};

// One work item: a tile of kTileCells cells against the runs
// [split * runs_per_split, ...) of the particles in batches
// [part * batches_per_part, ...) of the tile's particle order (job J).
// Called by all kDepositThreads threads of a workgroup.
// Lane (cell, group) = (lane % kTileCells, lane / kTileCells): the sixteen
// lanes of a wavefront's row hold different cells, so one ring update
// instruction touches different rings, and the four groups of a wavefront
// read their particles' records as LDS broadcasts.
// HOLD: which field a segment holds (0 the current state's, 1 the previous
// state's, 2 the linear interpolation between the two)
// G: bit 0 the far-field geometry, bit 1 potentials instead of fields
// DIV: the double slot coordinate divides (a divisor that fails the host check
// of canon_slot's corrections); a compile-time choice, so that the state loop
// carries no branch for it.
template <int M, int R, int G, int HOLD, int SH, bool DIV>
__device__ __forceinline__ void deposit_item(const DepositJob& J, int64_t tile, int64_t split,
                                             int64_t part, DepositShared<M, R, SH>& sh)
{
    constexpr int kTileCells = shape_cells(SH);  // this shape's tile, batch and run
    constexpr int kGroups = shape_groups(SH);
    constexpr int kRunL = shape_run(SH);
    constexpr bool FAR = (G & 1) != 0;
    constexpr bool POT = (G & 2) != 0;
    constexpr bool MIX = ModeTypes<M>::MIX;
    using T = typename ModeTypes<M>::T;
    using Acc = typename ModeTypes<M>::Acc;
    using Sink = CellSink<Acc, R>;
    using Rec = typename ModeTypes<M>::Rec;
    constexpr int RW = Sink::W;
    const Rec* recs = reinterpret_cast<const Rec*>(J.recs);

    const int tid = threadIdx.x;
    const int cl = tid % kTileCells;  // cell within the tile
    const int g = tid / kTileCells;   // particle group
    const int64_t row_i = tile * kTileCells + cl;  // internal (tile-ordered) cell row
    const bool active = row_i < J.n_c;
    const int n_t = (int)J.n_t;
    const Consts K{J.t0, J.inv_dt_det, J.inv_c, J.inv_c * J.inv_dt_det, J.dt_det, DIV};
    const double ntd = (double)n_t;
    // the time argument of the field and slot functions for state index sk: the
    // state time t_s (double mode, canonical rounding), or (t_s - t0) / dt_det
    const double ub0 = (J.t_first - J.t0) * J.inv_dt_det, dtu = J.dt * J.inv_dt_det;
    auto clock = [&](double sk) {
        if constexpr (MIX)
            return fma(sk, dtu, ub0);
        else
            return canon_state_time(J.t_first, sk, J.dt);
    };
    double xc[3] = {0.0, 0.0, 0.0};
    double fc[4] = {0.0, 0.0, 0.0, 1.0};  // far field: the cell's direction and distance
    RADIO_GLOBAL Acc* row = nullptr;
    if (active) {
        const RADIO_GLOBAL double* cells = gptr(J.cells);
        xc[0] = cells[3 * row_i];
        xc[1] = cells[3 * row_i + 1];
        xc[2] = cells[3 * row_i + 2];
        if constexpr (FAR) {
            const RADIO_GLOBAL double* f = gptr(J.far) + 4 * row_i;
            fc[0] = f[0];
            fc[1] = f[1];
            fc[2] = f[2];
            fc[3] = f[3];
        }
        row = gptr(reinterpret_cast<Acc*>(J.acc + row_i * J.n_t * 6));
    }
    const double Rinv = 1.0 / fc[3];
    // slot coordinate of a state, the same expression the field functions use
    auto slot_of = [&](const Rec& st, double tk) {
        if constexpr (FAR)
            return MIX ? slot_far_mixed(fc, st.x, tk, K) : slot_far_fp64(fc, st.x, tk, K);
        else
            return MIX ? slot_coord_mixed(xc, st.x, tk, K) : slot_coord_fp64(xc, st.x, tk, K);
    };
    RADIO_LDS double* my_ring = (RADIO_LDS double*)&sh.ring[cl * DepositShared<M, R, SH>::kStride];
    RADIO_LDS int* nb = (RADIO_LDS int*)&sh.nb[0][0];
    for (int i = g; i < R * RW; i += kGroups)
        my_ring[i] = 0.0;
    if (tid < kCounters)
        sh.cnt[tid] = 0;
    if (tid < 2 * kTileCells)
        nb[tid] = INT_MAX;
    int base = 0;  // the ring covers [base, base + R), 0 <= base <= max(n_t - R, 0)
    unsigned n_clip = 0, n_back = 0, n_bypass = 0;
    unsigned n_large = 0;  // large ring: the lane's segments (its interactions)
    // the tile's particle order for run rb (one order per group of runs)
    auto order_of = [&](int64_t rb_) {
        return gptr(J.perm + ((rb_ >> J.group_shift) * J.n_tiles + tile) * J.n_p);
    };
    const RADIO_GLOBAL double* charges = J.q ? gptr(J.q) : nullptr;
    const int64_t n_states = J.n_s + 1;
    const int64_t bt_begin = part * J.batches_per_part;
    const int64_t bt_end = min(bt_begin + J.batches_per_part, (J.n_p + kGroups - 1) / kGroups);
    const int64_t n_batches = bt_end - bt_begin;  // per run
    // The item's runs [rb_begin, rb_end), staged in parts of L segments: part
    // rb (states rb * L ... rb * L + L) of run rb / NS.
    constexpr int L = kSubRun<R, SH>;
    constexpr int NS = kRunL / L;
    const int64_t rb_begin = split * J.runs_per_split * NS;
    const int64_t rb_end =
        min(min(split * J.runs_per_split + J.runs_per_split, J.n_runs) * NS, (J.n_s + L - 1) / L);
    // The item's batches are taken part-major: part rb of the particles
    // order[bt * kGroups ...], bt = bt_begin .. bt_end - 1.
    // Before a batch is computed, one round of global loads brings its
    // records, its charges and the first positions of the next batch's
    // particles, whose lowest start slot per cell places the ring for that
    // batch before it is staged; the order entries these loads need were
    // fetched in the round before.
    auto advance = [&](int64_t& rb_, int64_t& bt_) {
        if (++bt_ == bt_end) {
            bt_ = bt_begin;
            ++rb_;
        }
    };
    // the lane's particle of batch (rb_, bt_), or -1 (the order of the part's run)
    auto lane_particle = [&](int64_t rb_, int64_t bt_, int lane_g) -> int {
        const int64_t i = bt_ * kGroups + lane_g;
        return (rb_ < rb_end && i < J.n_p) ? (int)order_of(rb_ / NS)[i] : -1;
    };
    // lowest start slot of the cell over a batch: the lane's particle starts at x
    // at state s_a (into nb[buf][cell])
    auto scout = [&](const double x[3], int64_t s_a, int buf) {
        const double t = canon_state_time(J.t_first, (double)(J.s0 + s_a), J.dt);
        double u;
        if constexpr (FAR) {
            u = (t + (fc[3] - (x[0] * fc[0] + x[1] * fc[1] + x[2] * fc[2])) * K.inv_c - K.t0) *
                K.inv_dt_det;
        } else {
            const double d0 = xc[0] - x[0], d1 = xc[1] - x[1], d2 = xc[2] - x[2];
            double dist, rinv;  // to ~1e-15: ample for placing the ring
            fast_norm(norm2_fast(d0, d1, d2), &dist, &rinv);
            u = (t + dist * K.inv_c - K.t0) * K.inv_dt_det;
        }
        if (u == u) {
            const int f = (int)floor(fmin(fmax(u, -1.0), (double)n_t + 1.0));
            __hip_atomic_fetch_min(nb + buf * kTileCells + cl, f, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    };
    auto first_position = [&](int p, int64_t s_a) {
        return gptr(reinterpret_cast<const double*>(recs + (int64_t)p * n_states + s_a));
    };

    // Move the ring to start at new_base: slots leaving it go to HBM.  The
    // cell's kGroups lanes share the work.
    auto move_ring = [&](int new_base) {
        if (active) {
            int lo = base, hi = base + R;  // slots to flush
            if (new_base > base && new_base < base + R)
                hi = new_base;
            for (int j = lo + g; j < hi; j += kGroups) {
                RADIO_LDS double* q = my_ring + ring_pos<R>(j) * RW;
                double a[RW];
                bool nz = false;
#pragma unroll
                for (int k = 0; k < RW; ++k) {
                    a[k] = q[k];
                    q[k] = 0.0;
                    nz |= (a[k] != 0.0);
                }
                if (nz && j < n_t) {
                    if constexpr (M == kModeMixTwoSum) {
                        // the slot's double sum as a compensated pair
                        float hi[6], lo[6];
#pragma unroll
                        for (int k = 0; k < 6; ++k) {
                            hi[k] = (float)a[k];
                            lo[k] = (float)(a[k] - (double)hi[k]);
                        }
                        global_add_pair(row, j, hi, lo);
                    } else {
                        global_add(row, j, a);
                    }
                }
            }
        }
        base = new_base;
    };

    // Staging of a batch's records.  Single-precision kernels load them from
    // HBM straight into LDS (no registers held for them, which keeps their
    // register count at five wavefronts per SIMD); the double kernel, whose LDS
    // allows four workgroups per CU anyway, stages through registers with
    // kStageLanes threads per particle, which takes fewer instructions.  In
    // the latter the thread index passes through an empty asm so that what is
    // derived from it is recomputed per batch instead of being held in
    // registers across the field loop.
    // Large-ring workgroups (two per CU: their LDS allows no more) have too
    // few neighbours to hide a batch's loads, so they prefetch: the next
    // batch's records, charges and first positions are loaded into registers
    // while the current batch is computed, and written to LDS after it.
    constexpr bool kPrefetch = (R == kRingLarge);
    constexpr bool kStageDirect = MIX && !kPrefetch;
    constexpr int kStageLanes = kDepositThreads / kGroups;
    int t_stage = tid;
    asm volatile("" : "+v"(t_stage));
    // register staging: a thread holds pieces r0, r0 + kStageLanes, ... of the
    // records of particle t_stage / kStageLanes of the batch (pieces of 16
    // bytes where the record size allows, else of 8)
    using Piece = typename std::conditional<sizeof(Rec) % 16 == 0, v2i64, long long>::type;
    constexpr int kPieces = (int)(sizeof(Rec) / sizeof(Piece));
    constexpr int kIter = ((L + 1) * kPieces + kStageLanes - 1) / kStageLanes;
    // the records (states s_a .. s_a + L, contiguous) and the charge of particle p
    auto load_records = [&](int p, int64_t s_a_, Piece(&v)[kIter], double& qs) {
        const int per = (int)(min((int64_t)L, J.n_s - s_a_) + 1) * kPieces;
        int t = t_stage;
        asm volatile("" : "+v"(t));
        const int r0 = t % kStageLanes;
        if (p >= 0) {
            const RADIO_GLOBAL Piece* src =
                gptr(reinterpret_cast<const Piece*>(recs + (int64_t)p * n_states + s_a_));
#pragma unroll
            for (int j = 0; j < kIter; ++j)
                if (r0 + j * kStageLanes < per)
                    v[j] = src[r0 + j * kStageLanes];
            if (r0 == 0)
                qs = charges ? charges[p] : -1.0;
        }
    };
    auto store_records = [&](int p, int len_, const Piece(&v)[kIter], double qs) {
        const int per = (len_ + 1) * kPieces;
        int t = t_stage;
        asm volatile("" : "+v"(t));
        const int gg = t / kStageLanes;
        const int r0 = t % kStageLanes;
        if (p >= 0) {
            Piece* dst = reinterpret_cast<Piece*>(&sh.rec[gg][0]);
#pragma unroll
            for (int j = 0; j < kIter; ++j)
                if (r0 + j * kStageLanes < per)
                    dst[r0 + j * kStageLanes] = v[j];
            if (r0 == 0)
                sh.sq[gg] = qs;
        }
    };
    int64_t rb = rb_begin, bt = bt_begin;  // the current batch
    int64_t rb1 = rb, bt1 = bt;     // the next one
    advance(rb1, bt1);
    int p_stage = -1, p_scout = -1;  // this thread's particle to stage; the lane's to scout
    int p_next = -1;                 // prefetch: this thread's particle of the next batch
    Piece v_pre[kPrefetch ? kIter : 1];  // prefetch: the records in flight
    double q_pre = 0.0;
    __syncthreads();  // rings and start slots cleared
    if (rb_begin < rb_end && n_batches > 0) {
        const int p0 = lane_particle(rb, bt, g);
        if (active && p0 >= 0) {
            const RADIO_GLOBAL double* x = first_position(p0, rb * L);
            const double xs[3] = {x[0], x[1], x[2]};
            scout(xs, rb * L, 0);
        }
        if constexpr (kStageDirect) {
            if (tid < kGroups)
                sh.ord[0][tid] = lane_particle(rb, bt, tid);
        } else {
            p_stage = lane_particle(rb, bt, t_stage / kStageLanes);
        }
        if constexpr (kPrefetch) {
            load_records(p_stage, rb * L, v_pre, q_pre);
            p_next = lane_particle(rb1, bt1, t_stage / kStageLanes);
        }
        p_scout = lane_particle(rb1, bt1, g);
    }
    __syncthreads();
    for (int buf = 0; rb < rb_end && n_batches > 0; buf ^= 1) {
        const int64_t s_a = rb * L;
        const int len = (int)min((int64_t)L, J.n_s - s_a);
        const int64_t i0 = bt * kGroups;
        const int np = (int)min((int64_t)kGroups, J.n_p - i0);
        // slide the ring to this batch's earliest start (every lane of the
        // previous batch is past the barrier that ended it)
        const int lo_slot = nb[buf * kTileCells + cl];
        if (lo_slot != INT_MAX) {
            const double mc = fmin(fmax((double)lo_slot - (double)kRingMargin, 0.0),
                                   fmax((double)(n_t - R), 0.0));
            const int nbase = (int)mc;
            if (nbase != base)
                move_ring(nbase);
        }
        int64_t rb2 = rb1, bt2 = bt1;  // the batch after the next
        advance(rb2, bt2);
        if constexpr (kStageDirect) {
            // The records go from HBM straight to LDS (16 bytes a lane, no
            // registers).  A wavefront stages whole rows: row gg (the run of
            // particle ord[gg], contiguous in HBM and in LDS) in rounds of 64
            // pieces, lane i taking piece h * 64 + i.  The particle is the same
            // for the whole wavefront, so the addressing is scalar but for the
            // lane's offset.  With the records, in the same round of loads: the
            // batch's charges, the order entries of the next batch and the next
            // batch's first positions for the ring.
            static_assert(sizeof(Rec) % 16 == 0, "records move in 16-byte pieces");
            constexpr int kPieces = (int)(sizeof(Rec) / 16);
            constexpr int kPer = (L + 1) * kPieces;  // pieces of a full row
            constexpr int kWaves = kDepositThreads / 64;
            constexpr int kRowsPerWave = kGroups / kWaves;
            constexpr int kHalves = (kPer + 63) / 64;  // rounds per row
            const int per = (len + 1) * kPieces;
            const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
            const int lane = tid % 64;
            RADIO_LDS char* rec_lds = (RADIO_LDS char*)&sh.rec[0][0];
            const RADIO_GLOBAL char* rec_hbm = reinterpret_cast<const RADIO_GLOBAL char*>(gptr(recs));
            int part[kRowsPerWave];  // the rows' particles, read before the first load writes LDS
#pragma unroll
            for (int k = 0; k < kRowsPerWave; ++k)
                part[k] = __builtin_amdgcn_readfirstlane(sh.ord[buf][wave + k * kWaves]);
#pragma unroll
            for (int k = 0; k < kRowsPerWave; ++k) {
                const int gg = wave + k * kWaves;
                if (gg < np) {
                    const RADIO_GLOBAL char* src =
                        rec_hbm + ((int64_t)part[k] * n_states + s_a) * (int64_t)sizeof(Rec);
#pragma unroll
                    for (int h = 0; h < kHalves; ++h)
                        if (h * 64 + lane < per)
                            __builtin_amdgcn_global_load_lds(src + (h * 64 + lane) * 16,
                                                             rec_lds + (gg * kPer + h * 64) * 16, 16,
                                                             0, 0);
                }
            }
            double qs = 0.0;
            if (tid < np)
                qs = charges ? charges[sh.ord[buf][tid]] : -1.0;
            const int ord_next = tid < kGroups ? lane_particle(rb1, bt1, tid) : -1;
            double xs[3] = {0.0, 0.0, 0.0};
            const bool scouting = active && p_scout >= 0;
            if (scouting) {
                const RADIO_GLOBAL double* x = first_position(p_scout, rb1 * L);
                xs[0] = x[0];
                xs[1] = x[1];
                xs[2] = x[2];
            }
            const int p_scout_next = lane_particle(rb2, bt2, g);
            if (tid < np)
                sh.sq[tid] = qs;
            if (tid < kGroups)
                sh.ord[buf ^ 1][tid] = ord_next;
            if (scouting)
                scout(xs, rb1 * L, buf ^ 1);
            p_scout = p_scout_next;
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the records are in LDS
        } else if constexpr (kPrefetch) {
            // this batch's records came into registers while the previous one was computed
            store_records(p_stage, len, v_pre, q_pre);
        } else {
            const int per = (len + 1) * kPieces;
            int t = t_stage;
            asm volatile("" : "+v"(t));
            const int gg = t / kStageLanes;
            const int r0 = t % kStageLanes;
            // one round of loads: the records of particle p_stage (states
            // s_a .. s_a + len, contiguous), its charge, the next batch's first
            // position for the lane, and the order entries of the next round
            Piece v[kIter];
            double qs = 0.0;
            if (p_stage >= 0) {
                const RADIO_GLOBAL Piece* src =
                    gptr(reinterpret_cast<const Piece*>(recs + (int64_t)p_stage * n_states + s_a));
#pragma unroll
                for (int j = 0; j < kIter; ++j)
                    if (r0 + j * kStageLanes < per)
                        v[j] = src[r0 + j * kStageLanes];
                if (r0 == 0)
                    qs = charges ? charges[p_stage] : -1.0;
            }
            double xs[3] = {0.0, 0.0, 0.0};
            const bool scouting = active && p_scout >= 0;
            if (scouting) {
                const RADIO_GLOBAL double* x = first_position(p_scout, rb1 * L);
                xs[0] = x[0];
                xs[1] = x[1];
                xs[2] = x[2];
            }
            const int p_stage_next = lane_particle(rb1, bt1, gg);
            const int p_scout_next = lane_particle(rb2, bt2, g);
            if (p_stage >= 0) {
                Piece* dst = reinterpret_cast<Piece*>(&sh.rec[gg][0]);
#pragma unroll
                for (int j = 0; j < kIter; ++j)
                    if (r0 + j * kStageLanes < per)
                        dst[r0 + j * kStageLanes] = v[j];
                if (r0 == 0)
                    sh.sq[gg] = qs;
            }
            if (scouting)
                scout(xs, rb1 * L, buf ^ 1);
            p_stage = p_stage_next;
            p_scout = p_scout_next;
        }
        if (tid < len + 1)
            sh.tk[tid] = clock((double)(J.s0 + s_a + tid));
        __syncthreads();
        if (tid < kTileCells)  // read by every lane before the barrier; next used two batches on
            nb[buf * kTileCells + tid] = INT_MAX;
        // prefetch: in flight while this batch is computed, the next batch's
        // records and charges, its first positions (for its ring placement) and
        // the order entries of the batch after it
        double xs_next[3] = {0.0, 0.0, 0.0};
        bool scout_next = false;
        int p_stage_after = -1, p_scout_after = -1;
        if constexpr (kPrefetch) {
            load_records(p_next, rb1 * L, v_pre, q_pre);
            scout_next = active && p_scout >= 0;
            if (scout_next) {
                const RADIO_GLOBAL double* x = first_position(p_scout, rb1 * L);
                xs_next[0] = x[0];
                xs_next[1] = x[1];
                xs_next[2] = x[2];
            }
            p_stage_after = lane_particle(rb2, bt2, t_stage / kStageLanes);
            p_scout_after = lane_particle(rb2, bt2, g);
        }
        if (active && g < np) {
            if constexpr (R == kRingLarge)
                n_large += (unsigned)len;
            Sink sink{my_ring, row, base, n_t, &n_bypass};
            const double q = sh.sq[g];
            // (the mixed records carry q/c in their betadot)
            const T qc = T(q * J.inv_c), qv = T(q * J.vscale), qv2 = T(2.0 * q * J.vscale);
            // the field of one staged state and its slot coordinate
            auto field_at = [&](const Rec& st, double tk, T F[6]) {
                if constexpr (POT) {
                    potentials_at<FAR>(xc, fc, st, q, F);
                    return slot_of(st, tk);
                } else if constexpr (FAR) {
                    if constexpr (MIX)
                        return field_far_mixed(fc, Rinv, st, tk, qv2, K, F);
                    else
                        return field_far_fp64(fc, Rinv, st, tk, qc, qv, K, F);
                } else {
                    if constexpr (MIX)
                        return field_mixed(xc, st, tk, qv2, K, F);
                    else
                        return field_fp64(xc, st, tk, qc, qv, K, F);
                }
            };
            T Fp[6];  // the previous state's field (HOLD != 0)
            double u_prev;
            if constexpr (HOLD != 0)
                u_prev = field_at(sh.rec[g][0], sh.tk[0], Fp);
            else
                u_prev = slot_of(sh.rec[g][0], sh.tk[0]);
            Carry<T> C;
            // open the slot where the run starts (a start far outside the window
            // leaves the first segment to the general path)
            const bool inside = u_prev >= -1.0 && u_prev < ntd + 1.0;
            carry_open(C, inside ? floor(u_prev) : (double)(INT_MIN / 2));
            C.lim = fast_limit(C.J1 - 1.0, u_prev, ntd);
            // segment k: the field of state k, held (or interpolated) over its arrivals
            auto segment = [&](const Rec& st, double tk) {
                T F[6];
                const double uk = field_at(st, tk, F);
                if constexpr (HOLD == 0) {
                    add_segment(C, sink, n_t, u_prev, uk, F, n_back, n_clip);
                } else {
                    if constexpr (HOLD == 1)
                        add_segment(C, sink, n_t, u_prev, uk, Fp, n_back, n_clip);
                    else
                        add_segment_linear(C, sink, n_t, u_prev, uk, Fp, F, n_back, n_clip);
#pragma unroll
                    for (int c = 0; c < 6; ++c)
                        Fp[c] = F[c];
                }
                u_prev = uk;
            };
            if constexpr (kPrefetch) {
                // the next state's record is read from LDS while this one is
                // worked on (two waves per SIMD hide little of the LDS latency)
                Rec cur = sh.rec[g][1];
                double t_cur = sh.tk[1];
                for (int k = 1; k <= len; ++k) {
                    const int kn = min(k + 1, len);
                    const Rec nxt = sh.rec[g][kn];
                    const double t_nxt = sh.tk[kn];
                    segment(cur, t_cur);
                    cur = nxt;
                    t_cur = t_nxt;
                }
            } else {
                for (int k = 1; k <= len; ++k)
                    segment(sh.rec[g][k], sh.tk[k]);
            }
            sink.flush((int)(C.J1 - 1.0), C.V);
        }
        if constexpr (kPrefetch) {
            if (scout_next)
                scout(xs_next, rb1 * L, buf ^ 1);
            p_stage = p_next;
            p_next = p_stage_after;
            p_scout = p_scout_after;
        }
        __syncthreads();  // records and rings are free for the next batch
        rb = rb1;
        bt = bt1;
        rb1 = rb2;
        bt1 = bt2;
    }
    move_ring(-1);  // flush what the ring still holds
    if (n_clip)
        atomicAdd(&sh.cnt[0], (unsigned long long)n_clip);
    if (n_back)
        atomicAdd(&sh.cnt[1], (unsigned long long)n_back);
    if (n_bypass)
        atomicAdd(&sh.cnt[2], (unsigned long long)n_bypass);
    if (n_large)
        atomicAdd(&sh.cnt[3], (unsigned long long)n_large);
    __syncthreads();
    if (tid < kCounters && sh.cnt[tid])
        __hip_atomic_fetch_add(gptr(J.counters) + tid, sh.cnt[tid], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

// deposit_item with the slot-coordinate form of the job (the single-precision
// modes have one)
template <int M, int R, int G, int HOLD, int SH>
__device__ __forceinline__ void deposit_item_of(const DepositJob& J, int64_t tile, int64_t split,
                                                int64_t part, DepositShared<M, R, SH>& sh)
{
    if constexpr (M == kModeF64) {
        if (J.slot_div)
            deposit_item<M, R, G, HOLD, SH, true>(J, tile, split, part, sh);
        else
            deposit_item<M, R, G, HOLD, SH, false>(J, tile, split, part, sh);
    } else {
        deposit_item<M, R, G, HOLD, SH, false>(J, tile, split, part, sh);
    }
}

// The work items item0 + [0, gridDim.x) of a single deposit, item =
// split * n_tiles + tile, one per workgroup (gridDim.x is a multiple of
// kXcds); items whose tile takes the other ring size leave at once.
// Waves per SIMD to ask of the register allocator.  A mixed-precision kernel with
// the small ring fits five wavefronts per SIMD in 96 VGPRs (its LDS allows five
// workgroups per CU).  For the exact-geometry, current-state kernel the
// allocator stays within that by itself and its own schedule is the faster
// one; the far-field, acceleration-only and held-field kernels go a few
// registers over, and keeping them at five waves (at the cost of a few spilled
// words in the hold kernels) is 4-6% faster on the undulator ensemble.  The
// double kernels are held to four workgroups per CU by their LDS; with both
// forms of the slot coordinate compiled in (see deposit_item_of) the default
// and previous-state kernels go a few registers over 128 by themselves and fit
// them on request (the previous-state hold with two spilled words), the linear
// hold would spill heavily and is left alone.  The other shapes: the 16-cell
// tile with runs of 8 segments has the LDS for five (single) or four (double)
// waves and is asked for them; the 8-cell tile's LDS allows three.
template <int M, int R, int G, int HOLD, int SH>
constexpr int kMinWaves =
    R != kRingSmall                      ? 1
    : SH == 1                            ? 1
    : M != kModeF64 && (G != 0 || HOLD != 0 || SH == 2) ? 5
    : M == kModeF64 && HOLD != 2         ? 4
                                         : 1;

template <int M, int R, int G, int HOLD, int SH>
__global__ __launch_bounds__(kDepositThreads)
__attribute__((amdgpu_waves_per_eu(kMinWaves<M, R, G, HOLD, SH>))) void deposit_kernel(
    DepositJob J, int64_t item0)
{
    __shared__ __align__(16) DepositShared<M, R, SH> sh;
    // Workgroups are dealt round-robin over the XCDs; give each XCD a contiguous
    // range of items, so that the workgroups resident on one XCD work on
    // neighbouring tiles of the same runs, whose records and particle orders
    // are alike, and share that XCD's L2.
    const int64_t per_xcd = (int64_t)gridDim.x / kXcds;
    const int64_t logical =
        item0 + (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
    if (logical >= J.n_tiles * J.n_splits * J.n_parts)
        return;
    const int64_t tile = logical % J.n_tiles;
    if (gptr(J.ring_sel)[tile] != (R == kRingLarge ? 1 : 0))
        return;
    const int64_t rest = logical / J.n_tiles;  // split-major, then part
    deposit_item_of<M, R, G, HOLD, SH>(J, tile, rest / J.n_parts, rest % J.n_parts, sh);
}

// Persistent workgroups for many independent deposits: each takes the next work
// item (largest first, as ordered by the host) from a device counter until
// the list is exhausted, so uneven jobs share one launch without a tail of idle
// workgroups; items whose tile takes the other ring size are skipped.  Every
// workgroup leaves once the counter passes n_items.
// (The persistent loop costs registers: every single-precision variant with the
// small ring goes over 96 VGPRs by itself, and five waves per SIMD, with a few
// spilled words, make the 64-set batched benchmark 1.2% faster; the double
// small-ring variants are asked for the four waves their LDS allows.)
template <int M, int R, int G, int HOLD, int SH>
constexpr int kPersistentWaves = R != kRingSmall || SH == 1           ? 1
                                 : M != kModeF64                      ? 5
                                 : HOLD != 2                          ? 4
                                                                      : 1;

template <int M, int R, int G, int HOLD, int SH>
__global__ __launch_bounds__(kDepositThreads)
__attribute__((amdgpu_waves_per_eu(kPersistentWaves<M, R, G, HOLD, SH>))) void
deposit_persistent_kernel(
    const DepositJob* __restrict__ jobs, const WorkItem* __restrict__ items, int64_t n_items,
    unsigned long long* __restrict__ next)
{
    __shared__ __align__(16) DepositShared<M, R, SH> sh;
    __shared__ int64_t cur;
    for (;;) {
        __syncthreads();  // everyone has read the previous `cur`
        if (threadIdx.x == 0)
            cur = (int64_t)atomicAdd(next, 1ull);
        __syncthreads();
        const int64_t it = cur;
        if (it >= n_items)
            break;
        const WorkItem w = items[it];
        const DepositJob J = jobs[w.job];
        if (gptr(J.ring_sel)[w.tile] != (R == kRingLarge ? 1 : 0))
            continue;
        deposit_item_of<M, R, G, HOLD, SH>(J, w.tile, w.split, w.part, sh);
    }
}

// E and B from the slot accumulator: E[c][j][0..2] and B[c][j][0..2] for the
// caller's cell index c of internal row r.  The compensated single
// accumulator holds (hi, lo) pairs, folded to double.  One thread per slot.
template <bool PAIRS>
__global__ __launch_bounds__(256) void readout_kernel(const double* __restrict__ acc, int64_t n_c,
                                                      int64_t n_t,
                                                      const int64_t* __restrict__ user_index,
                                                      double* __restrict__ E,
                                                      double* __restrict__ B)
{
    const int64_t total = n_c * n_t;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / n_t;
        const int64_t j = i - r * n_t;
        double v[6];
        if (PAIRS) {
            const float* q = reinterpret_cast<const float*>(acc) + i * 12;
#pragma unroll
            for (int k = 0; k < 6; ++k)
                v[k] = (double)q[k] + (double)q[6 + k];
        } else {
#pragma unroll
            for (int k = 0; k < 6; ++k)
                v[k] = acc[i * 6 + k];
        }
        const int64_t o = (user_index[r] * n_t + j) * 3;
        if (E) {
            E[o] = v[0];
            E[o + 1] = v[1];
            E[o + 2] = v[2];
        }
        if (B) {
            B[o] = v[3];
            B[o + 1] = v[4];
            B[o + 2] = v[5];
        }
    }
}

__global__ void zero_kernel(double* p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void zero_u64_kernel(unsigned long long* p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ void arrival_kernel(const double* cells, const double* pts, const double* t, int64_t n,
                               double inv_c, double* out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        double d0 = cells[3 * i] - pts[3 * i];
        double d1 = cells[3 * i + 1] - pts[3 * i + 1];
        double d2 = cells[3 * i + 2] - pts[3 * i + 2];
        out[i] = canon_arrival(t[i], canon_sqrt(canon_norm2(d0, d1, d2)), inv_c);
    }
}

// slot coordinates (t + |x_cell - x|/c - t0) / dt_det of explicit triples, as the
// double deposit rounds them
__global__ void slot_coord_kernel(const double* cells, const double* pts, const double* t,
                                  int64_t n, double inv_c, double t0, double dt_det,
                                  double inv_dt_det, int slot_div, double* out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        double d0 = cells[3 * i] - pts[3 * i];
        double d1 = cells[3 * i + 1] - pts[3 * i + 1];
        double d2 = cells[3 * i + 2] - pts[3 * i + 2];
        const double tau = canon_arrival(t[i], canon_sqrt(canon_norm2(d0, d1, d2)), inv_c);
        out[i] = canon_slot(tau, t0, dt_det, inv_dt_det, slot_div != 0);
    }
}

}  // namespace

constexpr int64_t kMaxDepositGrid = int64_t(1) << 22;  // workgroups of one deposit launch

void set_shape(DepositJob& job, int shape)
{
    job.shape = shape;
    job.tile_cells = shape_cells(shape);
    job.groups = shape_groups(shape);
    job.run_l = shape_run(shape);
}

void plan_job(DepositJob& job, int target_blocks, int64_t capacity)
{
    job.n_runs = (job.n_s + job.run_l - 1) / job.run_l;
    job.n_tiles = (job.n_c + job.tile_cells - 1) / job.tile_cells;
    int64_t splits = 1;
    if (target_blocks > 0) {
        splits = (target_blocks + job.n_tiles - 1) / job.n_tiles;
    } else {
        // short items (at least kMinItemBatches batches, so that an item's
        // set-up and final ring flush stay small), unless that leaves fewer
        // items than the device holds at once
        const int64_t n_batches = std::max<int64_t>((job.n_p + job.groups - 1) / job.groups, 1);
        const int64_t rps = std::max<int64_t>(1, (kMinItemBatches + n_batches - 1) / n_batches);
        splits = (job.n_runs + rps - 1) / rps;
        if (job.n_tiles * splits < capacity)
            splits = job.n_runs;
    }
    if (splits < 1)
        splits = 1;
    if (splits > job.n_runs)
        splits = job.n_runs;
    job.runs_per_split = (job.n_runs + splits - 1) / splits;
    job.n_splits = (job.n_runs + job.runs_per_split - 1) / job.runs_per_split;
    // few runs (a short chunk): ranges of the sorted particles as well
    const int64_t n_batches = std::max<int64_t>((job.n_p + job.groups - 1) / job.groups, 1);
    int64_t parts = 1;
    const int64_t items = job.n_tiles * job.n_splits;
    if (target_blocks <= 0 && items < 2 * capacity) {
        parts = (2 * capacity + items - 1) / items;
        parts = std::max<int64_t>(1, std::min<int64_t>(parts, n_batches / 16));
    }
    set_parts(job, parts);
}

int64_t max_order_groups(const DepositJob& job, size_t rec_bytes, int64_t budget_mib)
{
    const double per_group = (double)job.n_tiles * (double)job.n_p * sizeof(int32_t);
    const double budget =
        budget_mib > 0 ? (double)budget_mib * (double)(int64_t(1) << 20)
                       : std::max((double)(job.n_s + 1) * (double)job.n_p * (double)rec_bytes,
                                  (double)(int64_t(1) << 30));
    return (int64_t)std::max(1.0, std::min(budget / per_group, (double)INT32_MAX));
}

void set_groups(DepositJob& job, int64_t max_groups)
{
    int64_t groups = std::min(job.n_runs, std::max<int64_t>(1, max_groups));
    // a few batches gain nothing from re-sorting, and each order costs a histogram
    if (job.n_p < min_group_particles(job))
        groups = 1;
    groups = std::max<int64_t>(1, groups);
    const int64_t want = (job.n_runs + groups - 1) / groups;
    job.group_shift = 0;
    while ((int64_t(1) << job.group_shift) < want)
        ++job.group_shift;
    job.runs_per_group = int64_t(1) << job.group_shift;
    job.n_groups = (job.n_runs + job.runs_per_group - 1) / job.runs_per_group;
}

void set_parts(DepositJob& job, int64_t parts)
{
    const int64_t n_batches = std::max<int64_t>((job.n_p + job.groups - 1) / job.groups, 1);
    parts = std::max<int64_t>(1, std::min<int64_t>(parts, n_batches));
    job.batches_per_part = (n_batches + parts - 1) / parts;
    job.n_parts = (n_batches + job.batches_per_part - 1) / job.batches_per_part;
}

hipError_t launch_zero(double* p, int64_t n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192)
        blocks = 8192;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_kinematics(const DepositJob& job, int mode, hipStream_t s)
{
    const int64_t total = job.n_p * (job.n_s + 1);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536)
        blocks = 65536;
    const int rule = job.hold == 2 ? kBdCentred : (job.hold == 1 ? kBdBackwardFirst : kBdBackward);
    if (mode == kModeF64)
        hipLaunchKernelGGL(kinematics_kernel<kModeF64>, dim3((unsigned)blocks), dim3(256), 0, s,
                           job.x, job.u, job.q, job.n_p, job.n_s, job.xs_stride, -job.s_before,
                           job.n_s + job.s_after, job.dt, job.inv_c, rule, job.recs);
    else
        hipLaunchKernelGGL(kinematics_kernel<kModeMix>, dim3((unsigned)blocks), dim3(256), 0, s,
                           job.x, job.u, job.q, job.n_p, job.n_s, job.xs_stride, -job.s_before,
                           job.n_s + job.s_after, job.dt, job.inv_c, rule, job.recs);
    return hipGetLastError();
}

hipError_t launch_order(const DepositJob& job, hipStream_t s)
{
    hipLaunchKernelGGL(order_kernel, dim3((unsigned)(job.n_tiles * job.n_groups)), dim3(256), 0, s,
                       job.x, job.n_p, job.n_s, job.xs_stride, job.n_tiles,
                       (int64_t)job.tile_cells, job.runs_per_group * job.run_l,
                       job.cells, job.n_c, job.inv_c, job.inv_dt_det, job.perm);
    return hipGetLastError();
}

hipError_t launch_ring_choice(const DepositJob& job, int mode, hipStream_t s)
{
    if (job.n_tiles <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(ring_choice_kernel, dim3((unsigned)job.n_tiles), dim3(256), 0, s,
                       reinterpret_cast<const char*>(job.recs), (int64_t)rec_bytes(mode),
                       job.perm, job.n_tiles, job.runs_per_group, job.cells, job.far, job.n_c,
                       job.n_p, job.n_s, job.n_runs,
                       job.t_first,
                       job.s0, job.dt, job.t0, job.inv_dt_det, job.inv_c, job.n_t,
                       (int)job.tile_cells, (int)job.groups, (int)job.run_l, job.ring_sel);
    return hipGetLastError();
}

// kernel variants (kernel_variant): precision mode x geometry/quantity (far
// field, potentials) x hold rule for the default shape; precision mode for the
// other shapes with the default options; each with both ring sizes
template <int V>
struct VariantOf {
    static constexpr bool kOpt = V < kOptionVariants;
    static constexpr int M = kOpt ? V % 3 : (V - kOptionVariants) % 3;
    static constexpr int G = kOpt ? (V / 3) % 4 : 0;
    static constexpr int HOLD = kOpt ? V / 12 : 0;
    static constexpr int SH = kOpt ? 0 : 1 + (V - kOptionVariants) / 3;
};

template <int V>
static void launch_deposit_index(const DepositJob& job, dim3 grid, hipStream_t s)
{
    using K = VariantOf<V>;
    // more items than one launch holds run in several launches
    const int64_t n_items = job.n_tiles * job.n_splits * job.n_parts;
    for (int64_t item0 = 0; item0 < n_items; item0 += grid.x)
        hipLaunchKernelGGL((deposit_kernel<K::M, kRingSmall, K::G, K::HOLD, K::SH>), grid,
                           dim3(kDepositThreads), 0, s, job, item0);
    for (int64_t item0 = 0; item0 < n_items; item0 += grid.x)
        hipLaunchKernelGGL((deposit_kernel<K::M, kRingLarge, K::G, K::HOLD, K::SH>), grid,
                           dim3(kDepositThreads), 0, s, job, item0);
}

template <int V>
static void launch_persistent_index(const DepositJob* jobs, const WorkItem* items,
                                    int64_t n_items, unsigned long long* next, int blocks_small,
                                    int blocks_large, hipStream_t s)
{
    using K = VariantOf<V>;
    hipLaunchKernelGGL((deposit_persistent_kernel<K::M, kRingSmall, K::G, K::HOLD, K::SH>),
                       dim3((unsigned)blocks_small), dim3(kDepositThreads), 0, s, jobs, items,
                       n_items, next);
    hipLaunchKernelGGL((deposit_persistent_kernel<K::M, kRingLarge, K::G, K::HOLD, K::SH>),
                       dim3((unsigned)blocks_large), dim3(kDepositThreads), 0, s, jobs, items,
                       n_items, next + 1);
}

template <int V>
static int blocks_per_cu_index(bool large_ring)
{
    int n = 0;
    using K = VariantOf<V>;
    const void* f =
        large_ring
            ? reinterpret_cast<const void*>(
                  deposit_persistent_kernel<K::M, kRingLarge, K::G, K::HOLD, K::SH>)
            : reinterpret_cast<const void*>(
                  deposit_persistent_kernel<K::M, kRingSmall, K::G, K::HOLD, K::SH>);
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kDepositThreads, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

template <int... V>
struct VariantTable {
    using Single = void (*)(const DepositJob&, dim3, hipStream_t);
    using Launch = void (*)(const DepositJob*, const WorkItem*, int64_t, unsigned long long*,
                            int, int, hipStream_t);
    using Occ = int (*)(bool);
    static constexpr Single single[] = {&launch_deposit_index<V>...};
    static constexpr Launch launch[] = {&launch_persistent_index<V>...};
    static constexpr Occ occupancy[] = {&blocks_per_cu_index<V>...};
};
template <int... V>
constexpr VariantTable<V...> make_table(std::integer_sequence<int, V...>)
{
    return {};
}
using Variants = decltype(make_table(std::make_integer_sequence<int, kKernelVariants>{}));

hipError_t launch_deposit(const DepositJob& job, int mode, int64_t max_grid, hipStream_t s)
{
    int64_t blocks = job.n_tiles * job.n_splits * job.n_parts;
    if (blocks <= 0)
        return hipSuccess;
    blocks = (blocks + kXcds - 1) / kXcds * kXcds;  // a multiple of the XCD count
    // more items than max_grid (and kMaxDepositGrid) run in several launches
    const int64_t cap = std::max<int64_t>(kXcds, std::min<int64_t>(max_grid, kMaxDepositGrid));
    blocks = std::min<int64_t>(blocks, cap / kXcds * kXcds);
    const int v = kernel_variant(mode, job);
    if (v < 0 || v >= kKernelVariants)
        return hipErrorInvalidValue;
    Variants::single[v](job, dim3((unsigned)blocks), s);
    return hipGetLastError();
}

hipError_t launch_deposit_batch(const DepositJob* jobs, const WorkItem* items, int64_t n_items,
                                unsigned long long* next, int variant, int blocks_small,
                                int blocks_large, hipStream_t s)
{
    if (n_items <= 0)
        return hipSuccess;
    if (variant < 0 || variant >= kKernelVariants)
        return hipErrorInvalidValue;
    hipError_t e = launch_zero_u64(next, 2, s);
    if (e != hipSuccess)
        return e;
    Variants::launch[variant](jobs, items, n_items, next, blocks_small, blocks_large, s);
    return hipGetLastError();
}

int persistent_blocks_per_cu(int variant, bool large_ring)
{
    if (variant < 0 || variant >= kKernelVariants)
        return 1;
    // a property of the code object: asked once per kernel
    static std::atomic<int> known[kKernelVariants][2];
    const int r = large_ring ? 1 : 0;
    int n = known[variant][r].load(std::memory_order_relaxed);
    if (n <= 0) {
        n = Variants::occupancy[variant](large_ring);
        known[variant][r].store(n, std::memory_order_relaxed);
    }
    return n;
}

hipError_t launch_readout(const double* acc, int64_t n_c, int64_t n_t, const int64_t* user_index,
                          bool pairs, double* E, double* B, hipStream_t s)
{
    if (n_c <= 0)
        return hipSuccess;
    int64_t blocks = (n_c * n_t + 255) / 256;
    if (blocks > 65536)
        blocks = 65536;
    if (pairs)
        hipLaunchKernelGGL(readout_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, acc, n_c,
                           n_t, user_index, E, B);
    else
        hipLaunchKernelGGL(readout_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, acc, n_c,
                           n_t, user_index, E, B);
    return hipGetLastError();
}

hipError_t launch_arrival(const double* cells, const double* pts, const double* t, int64_t n,
                          double inv_c, double* out, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(arrival_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cells,
                       pts, t, n, inv_c, out);
    return hipGetLastError();
}

hipError_t launch_slot_coords(const double* cells, const double* pts, const double* t, int64_t n,
                              double inv_c, double t0, double dt_det, double inv_dt_det,
                              bool slot_div, double* out, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(slot_coord_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cells,
                       pts, t, n, inv_c, t0, dt_det, inv_dt_det, slot_div ? 1 : 0, out);
    return hipGetLastError();
}

}  // namespace radio
