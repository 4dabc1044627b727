// HIP kernels of libradio for gfx950 (MI355X).
//
// The deposit evaluates, for every (particle, segment, cell) triple, the
// Lienard-Wiechert field (Eq. 1) of the segment's current state and the
// arrival times of its two end states (Eq. 2), and adds the field held
// between those arrival times to the detector slots with the integrator
// weights of Sec. 3.2 / Alg. 2.
//
// Slot-difference accumulator.  The detector stores, per cell and slot, the
// difference between consecutive slot values; the readout turns differences
// back into slot values with a prefix sum along the slots.  A lane walks one
// particle's segments in order and integrates the held field over its current
// slot with the exact slot-unit overlaps of Alg. 2; it emits a difference only
// when the particle's arrivals move to a later slot.  A segment spanning many
// slots therefore costs two emissions (its value is constant in between), and
// consecutive segments landing in the same slot are summed in registers
// before any memory traffic.
//
// Work decomposition.  One lane owns one detector cell (256 cells per
// workgroup, 4 wavefronts).  Trajectories are cut into runs of kRunL
// segments; a tile of kTileP particles x (kRunL + 1) states is staged in LDS
// (coalesced SoA loads, kinematics computed once per state) and every lane
// walks the tile's states in order against its own cell, so the state data
// is a wave-uniform LDS broadcast.  Runs are independent: a run of kRunL
// segments needs its kRunL + 1 end states, so the state two runs share is
// staged (and its arrival time evaluated) by both, and each segment belongs
// to exactly one run.  Workgroups along the second grid dimension take
// contiguous ranges of (run, particle block) tiles, so the same cells receive
// deposits from several workgroups and the detector is updated with atomic
// adds.
#include "radio_internal.h"

#include <type_traits>

namespace radio {

namespace {

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

__device__ __forceinline__ double canon_state_time(double t_first, int64_t s, double dt)
{
#pragma clang fp contract(off)
    return t_first + (double)s * dt;
}

__device__ __forceinline__ double canon_arrival(double t, double R, double inv_c)
{
#pragma clang fp contract(off)
    return t + R * inv_c;
}

// slot coordinate (t_det - t0) / dt_det, as a product with 1/dt_det
__device__ __forceinline__ double canon_slot(double tau, double t0, double inv_dt_det)
{
#pragma clang fp contract(off)
    return (tau - t0) * inv_dt_det;
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

// ---------------------------------------------------------------------------

struct StateRec {           // one staged trajectory state (96 B, 16-B aligned)
    double x[3];
    double b[3];
    double bd[3];
    double g2i;
    float bdf[3];           // betadot and 1/gamma^2 rounded to single for the mixed field
    float g2if;
};

// Where a lane's finished slot differences go.  Double path: one atomic add per
// component.  Mixed path: a compensated single-precision pair (hi, lo) per
// component; the atomic add on hi returns the old value, so the lane knows the
// exact sum the hardware rounded (old + v) and adds that rounding error
// (two-sum) to lo.
struct RowF64 {
    double* p;  // [n_t][6]
    __device__ __forceinline__ void flush(int n_t, int j, const double a[6]) const
    {
        if (j >= 0 && j < n_t) {
            double* q = p + (int64_t)j * 6;
#pragma unroll
            for (int k = 0; k < 6; ++k)
                unsafeAtomicAdd(q + k, a[k]);
        }
    }
};

__device__ __forceinline__ float two_sum_err(float a, float b, float s)
{
#pragma clang fp contract(off)
    const float bv = s - a;
    return (a - (s - bv)) + (b - bv);
}

struct RowMixed {
    float* p;  // [n_t][12]: hi[6] then lo[6]
    __device__ __forceinline__ void flush(int n_t, int j, const float a[6]) const
    {
        if (j >= 0 && j < n_t) {
            float* q = p + (int64_t)j * 12;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const float old = atomicAdd(q + k, a[k]);
                unsafeAtomicAdd(q + 6 + k, two_sum_err(old, a[k], old + a[k]));
            }
        }
    }
};

// A lane's open slot.  For the run being processed the lane integrates the
// held field over its current slot J (V) and remembers the previous slot's
// value (Vp); when the run leaves slot J the difference V - Vp is final and
// goes to the detector, so every emitted number is a slot value difference,
// with the same exact slot-unit overlaps as the integrator definition.
template <typename T>
struct Carry {
    int J;                  // current slot, -1 when nothing is open
    T V[6];                 // integral of the held field over slot J so far
    T Vp[6];                // this run's value in slot J - 1
};

template <typename T>
__device__ __forceinline__ void carry_init(Carry<T>& C)
{
    C.J = -1;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        C.V[k] = T(0);
        C.Vp[k] = T(0);
    }
}

// Finish the open slot: its value difference, then the drop to zero after it.
template <typename T, typename Row>
__device__ __forceinline__ void carry_close(Carry<T>& C, const Row& row, int n_t)
{
    if (C.J >= 0) {
        T d[6], m[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            d[k] = C.V[k] - C.Vp[k];
            m[k] = -C.V[k];
        }
        row.flush(n_t, C.J, d);
        row.flush(n_t, C.J + 1, m);
    }
    carry_init(C);
}

// Hold F over the slot-coordinate interval between a and b (Alg. 2: each slot
// receives F times its overlap with the interval, in units of dt_det; parts
// outside [0, n_t) are dropped).  Segments normally continue where the last
// one ended; any other start (a reversed or out-of-order segment) closes the
// open slot and opens a new one, which is exact because deposits add.
template <typename T, typename Row>
__device__ __forceinline__ void add_segment(Carry<T>& C, const Row& row, int n_t, double a,
                                            double b, const T F[6])
{
    const double ntd = (double)n_t;
    const double lo = fmin(fmax(fmin(a, b), 0.0), ntd);
    const double hi = fmin(fmax(fmax(a, b), 0.0), ntd);
    if (!(lo < hi))  // empty, entirely outside, or NaN
        return;
    const int jl = (int)floor(lo);  // lo < n_t
    const int jh = (int)floor(hi);  // <= n_t; n_t only when hi reaches the end
    if (jl != C.J) {
        carry_close(C, row, n_t);
        C.J = jl;
    }
    if (jh == C.J) {
        const T w = T(hi - lo);
#pragma unroll
        for (int k = 0; k < 6; ++k)
            C.V[k] += F[k] * w;
        return;
    }
    T d[6];
    const T wa = T((double)(C.J + 1) - lo);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        C.V[k] += F[k] * wa;
        d[k] = C.V[k] - C.Vp[k];
        C.Vp[k] = C.V[k];
    }
    row.flush(n_t, C.J, d);
    if (jh > C.J + 1) {  // whole slots in between hold F
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            d[k] = F[k] - C.Vp[k];
            C.Vp[k] = F[k];
        }
        row.flush(n_t, C.J + 1, d);
    }
    const T wb = T(hi - (double)jh);
#pragma unroll
    for (int k = 0; k < 6; ++k)
        C.V[k] = F[k] * wb;
    C.J = jh;
}

struct Consts {
    double t0, inv_dt_det, inv_c;
    float inv_cf;
};

// Lienard-Wiechert E, B (Eq. 1) at a cell from one staged state, all in double;
// returns the state's slot coordinate.  Everything after the canonical part may
// use FMAs.
__device__ __forceinline__ double field_fp64(const double xc[3], const StateRec& st, double t_s,
                                             double q, const Consts& K, double F[6])
{
    double d[3] = {xc[0] - st.x[0], xc[1] - st.x[1], xc[2] - st.x[2]};
    double R2 = canon_norm2(d[0], d[1], d[2]);
    double R = __builtin_sqrt(R2);
    double tau = canon_arrival(t_s, R, K.inv_c);
    double rinv = 1.0 / R;
    double n[3], w[3];
    canon_direction(d, rinv, st.b, n, w);
    double kap = canon_kappa(w, st.g2i);
    double k3inv = 1.0 / (kap * kap * kap);
    double ca = q * k3inv * rinv * K.inv_c;        // (q/c) / (kappa^3 R)
    double cv = q * st.g2i * k3inv * rinv * rinv;  // q / (gamma^2 kappa^3 R^2)
    // w x betadot, then n x (w x betadot)
    double a0 = w[1] * st.bd[2] - w[2] * st.bd[1];
    double a1 = w[2] * st.bd[0] - w[0] * st.bd[2];
    double a2 = w[0] * st.bd[1] - w[1] * st.bd[0];
    double m0 = n[1] * a2 - n[2] * a1;
    double m1 = n[2] * a0 - n[0] * a2;
    double m2 = n[0] * a1 - n[1] * a0;
    double E0 = cv * w[0] + ca * m0;
    double E1 = cv * w[1] + ca * m1;
    double E2 = cv * w[2] + ca * m2;
    F[0] = E0;
    F[1] = E1;
    F[2] = E2;
    F[3] = n[1] * E2 - n[2] * E1;
    F[4] = n[2] * E0 - n[0] * E2;
    F[5] = n[0] * E1 - n[1] * E0;
    return canon_slot(tau, K.t0, K.inv_dt_det);
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

// The mixed-precision field: double for what cancels (arrival time, slot
// coordinate, n - beta and kappa), single for the rest of Eq. 1.
__device__ __forceinline__ double field_mixed(const double xc[3], const StateRec& st, double t_s,
                                              float q, const Consts& K, float F[6])
{
    double d[3] = {xc[0] - st.x[0], xc[1] - st.x[1], xc[2] - st.x[2]};
    double R2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double R, rinv;
    fast_norm(R2, &R, &rinv);
    const double u = canon_slot(t_s + R * K.inv_c, K.t0, K.inv_dt_det);
    double nd[3] = {d[0] * rinv, d[1] * rinv, d[2] * rinv};
    double wd[3] = {nd[0] - st.b[0], nd[1] - st.b[1], nd[2] - st.b[2]};
    const double kap = 0.5 * ((wd[0] * wd[0] + wd[1] * wd[1] + wd[2] * wd[2]) + st.g2i);
    const float n[3] = {(float)nd[0], (float)nd[1], (float)nd[2]};
    const float w[3] = {(float)wd[0], (float)wd[1], (float)wd[2]};
    const float kinv = __builtin_amdgcn_rcpf((float)kap);
    const float k3inv = kinv * kinv * kinv;
    const float rinvf = (float)rinv;
    const float ca = q * k3inv * rinvf * K.inv_cf;
    const float cv = q * st.g2if * k3inv * rinvf * rinvf;
    const float a0 = w[1] * st.bdf[2] - w[2] * st.bdf[1];
    const float a1 = w[2] * st.bdf[0] - w[0] * st.bdf[2];
    const float a2 = w[0] * st.bdf[1] - w[1] * st.bdf[0];
    const float m0 = n[1] * a2 - n[2] * a1;
    const float m1 = n[2] * a0 - n[0] * a2;
    const float m2 = n[0] * a1 - n[1] * a0;
    const float E0 = cv * w[0] + ca * m0;
    const float E1 = cv * w[1] + ca * m1;
    const float E2 = cv * w[2] + ca * m2;
    F[0] = E0;
    F[1] = E1;
    F[2] = E2;
    F[3] = n[1] * E2 - n[2] * E1;
    F[4] = n[2] * E0 - n[0] * E2;
    F[5] = n[0] * E1 - n[1] * E0;
    return u;
}

__device__ __forceinline__ double slot_coord_fp64(const double xc[3], const StateRec& st,
                                                  double t_s, const Consts& K)
{
    double d[3] = {xc[0] - st.x[0], xc[1] - st.x[1], xc[2] - st.x[2]};
    double R = __builtin_sqrt(canon_norm2(d[0], d[1], d[2]));
    double tau = canon_arrival(t_s, R, K.inv_c);
    return canon_slot(tau, K.t0, K.inv_dt_det);
}

__device__ __forceinline__ double slot_coord_mixed(const double xc[3], const StateRec& st,
                                                   double t_s, const Consts& K)
{
    double d[3] = {xc[0] - st.x[0], xc[1] - st.x[1], xc[2] - st.x[2]};
    double R, rinv;
    fast_norm(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], &R, &rinv);
    return canon_slot(t_s + R * K.inv_c, K.t0, K.inv_dt_det);
}

// Stage the states s_a .. s_a+len of particles p0 .. p0+np-1 into LDS.
__device__ __forceinline__ void stage_tile(const DepositJob& J, StateRec (*rec)[kRunL + 1],
                                           double* sq, int64_t s_a, int len, int64_t p0, int np)
{
    const int tid = threadIdx.x;
    const int64_t stride = (J.n_s + 1) * J.n_p;
    for (int i = tid; i < kTileP * (kRunL + 1); i += kCellsPerBlock) {
        const int pp = i % kTileP;
        const int k = i / kTileP;
        if (pp < np && k <= len) {
            const int64_t off = (s_a + k) * J.n_p + (p0 + pp);
            StateRec& r = rec[pp][k];
            r.x[0] = J.x[off];
            r.x[1] = J.x[off + stride];
            r.x[2] = J.x[off + 2 * stride];
            canon_kinematics(J.u[off], J.u[off + stride], J.u[off + 2 * stride], r.b, &r.g2i);
            r.g2if = (float)r.g2i;
        }
    }
    if (tid < kTileP)
        sq[tid] = (tid < np) ? (J.q ? J.q[p0 + tid] : -1.0) : 0.0;
    __syncthreads();
    for (int i = tid; i < kTileP * kRunL; i += kCellsPerBlock) {
        const int pp = i % kTileP;
        const int k = 1 + i / kTileP;
        if (pp < np && k <= len) {
            StateRec& r = rec[pp][k];
            const StateRec& rp = rec[pp][k - 1];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                r.bd[c] = (r.b[c] - rp.b[c]) / J.dt;
                r.bdf[c] = (float)r.bd[c];
            }
        }
    }
    __syncthreads();
}

// One particle's run against one cell: the fields of states 1..len, each held
// between the arrival times of its segment's two end states.
template <bool MIX>
__device__ __forceinline__ void run_particle(const double xc[3], const StateRec* st, int len,
                                             int64_t s_a, double q, const DepositJob& J,
                                             const Consts& K, double* acc_row, int n_t,
                                             unsigned& n_clip, unsigned& n_back)
{
    using T = typename std::conditional<MIX, float, double>::type;
    using Row = typename std::conditional<MIX, RowMixed, RowF64>::type;
    Row row{reinterpret_cast<T*>(acc_row)};
    Carry<T> C;
    carry_init(C);
    const double t_a = canon_state_time(J.t_first, s_a, J.dt);
    double u_prev = MIX ? slot_coord_mixed(xc, st[0], t_a, K) : slot_coord_fp64(xc, st[0], t_a, K);
    for (int k = 1; k <= len; ++k) {
        T F[6];
        const double t_s = canon_state_time(J.t_first, s_a + k, J.dt);
        double uk;
        if constexpr (MIX)
            uk = field_mixed(xc, st[k], t_s, (float)q, K, F);
        else
            uk = field_fp64(xc, st[k], t_s, q, K, F);
        const bool back = uk < u_prev;
        n_back += back ? 1u : 0u;
        n_clip += (fmin(uk, u_prev) < 0.0 || fmax(uk, u_prev) > (double)n_t) ? 1u : 0u;
        add_segment(C, row, n_t, u_prev, uk, F);
        u_prev = uk;
    }
    carry_close(C, row, n_t);
}

template <bool MIX>
__global__ __launch_bounds__(kCellsPerBlock) void deposit_kernel(DepositJob J)
{
    __shared__ StateRec rec[kTileP][kRunL + 1];
    __shared__ double sq[kTileP];
    __shared__ unsigned long long s_cnt[2];

    const int tid = threadIdx.x;
    const int64_t cb = blockIdx.x % J.cell_blocks;
    const int64_t split = blockIdx.x / J.cell_blocks;
    const int64_t cell = cb * kCellsPerBlock + tid;
    const bool active = cell < J.n_c;
    const int n_t = (int)J.n_t;
    const Consts K{J.t0, J.inv_dt_det, J.inv_c, (float)J.inv_c};
    double xc[3] = {0.0, 0.0, 0.0};
    double* row = nullptr;
    if (active) {
        xc[0] = J.cells[3 * cell];
        xc[1] = J.cells[3 * cell + 1];
        xc[2] = J.cells[3 * cell + 2];
        row = J.acc + cell * J.n_t * 6;  // 6 doubles or 12 floats per slot
    }
    if (tid < 2)
        s_cnt[tid] = 0;
    unsigned n_clip = 0, n_back = 0;

    const int64_t tile_begin = split * J.tiles_per_split;
    const int64_t tile_end = min(tile_begin + J.tiles_per_split, J.n_tiles);
    for (int64_t tile = tile_begin; tile < tile_end; ++tile) {
        const int64_t run = tile / J.n_pb;
        const int64_t pb = tile - run * J.n_pb;
        const int64_t s_a = run * kRunL;
        const int len = (int)min((int64_t)kRunL, J.n_s - s_a);
        const int64_t p0 = pb * kTileP;
        const int np = (int)min((int64_t)kTileP, J.n_p - p0);
        __syncthreads();  // the previous tile's readers are done with the LDS
        stage_tile(J, rec, sq, s_a, len, p0, np);
        if (active) {
            for (int pp = 0; pp < np; ++pp)
                run_particle<MIX>(xc, rec[pp], len, s_a, sq[pp], J, K, row, n_t, n_clip, n_back);
        }
    }
    if (n_clip)
        atomicAdd(&s_cnt[0], (unsigned long long)n_clip);
    if (n_back)
        atomicAdd(&s_cnt[1], (unsigned long long)n_back);
    __syncthreads();
    if (tid < 2 && s_cnt[tid])
        atomicAdd(&J.counters[tid], s_cnt[tid]);
}

// Prefix sum of the slot differences along the slots of each cell; writes
// E[c][j][0..2] and B[c][j][0..2].  One workgroup per cell.  The mixed
// accumulator holds (hi, lo) single pairs, folded to double before the sum.
template <bool MIX>
__global__ __launch_bounds__(256) void readout_kernel(const double* __restrict__ acc, int64_t n_t,
                                                      double* __restrict__ E,
                                                      double* __restrict__ B)
{
    __shared__ double wsum[4][6];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t cell = blockIdx.x;
    const double* rowp = acc + cell * n_t * 6;
    const float* rowf = reinterpret_cast<const float*>(rowp);
    double carry[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t base = 0; base < n_t; base += 256) {
        const int64_t j = base + tid;
        double v[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            if (j < n_t)
                v[k] = MIX ? (double)rowf[j * 12 + k] + (double)rowf[j * 12 + 6 + k]
                           : rowp[j * 6 + k];
            else
                v[k] = 0.0;
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                double t = __shfl_up(v[k], off, 64);
                if (lane >= off)
                    v[k] += t;
            }
        }
        if (lane == 63) {
#pragma unroll
            for (int k = 0; k < 6; ++k)
                wsum[wave][k] = v[k];
        }
        __syncthreads();
        double tot[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            double pre = carry[k];
            for (int w = 0; w < wave; ++w)
                pre += wsum[w][k];
            v[k] += pre;
            tot[k] = carry[k] + ((wsum[0][k] + wsum[1][k]) + (wsum[2][k] + wsum[3][k]));
        }
        if (j < n_t) {
            const int64_t o = (cell * n_t + j) * 3;
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
#pragma unroll
        for (int k = 0; k < 6; ++k)
            carry[k] = tot[k];
        __syncthreads();
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
        out[i] = canon_arrival(t[i], __builtin_sqrt(canon_norm2(d0, d1, d2)), inv_c);
    }
}

}  // namespace

void plan_job(DepositJob& job, int target_blocks)
{
    const int64_t n_runs = (job.n_s + kRunL - 1) / kRunL;
    job.n_pb = (job.n_p + kTileP - 1) / kTileP;
    job.n_tiles = n_runs * job.n_pb;
    job.cell_blocks = (job.n_c + kCellsPerBlock - 1) / kCellsPerBlock;
    int64_t splits = (target_blocks + job.cell_blocks - 1) / job.cell_blocks;
    if (splits < 1)
        splits = 1;
    if (splits > job.n_tiles)
        splits = job.n_tiles;
    job.tiles_per_split = (job.n_tiles + splits - 1) / splits;
    job.n_splits = (job.n_tiles + job.tiles_per_split - 1) / job.tiles_per_split;
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

hipError_t launch_deposit_fp64(const DepositJob& job, hipStream_t s)
{
    const int64_t blocks = job.cell_blocks * job.n_splits;
    if (blocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(deposit_kernel<false>, dim3((unsigned)blocks), dim3(kCellsPerBlock), 0, s,
                       job);
    return hipGetLastError();
}

hipError_t launch_deposit_mixed(const DepositJob& job, hipStream_t s)
{
    const int64_t blocks = job.cell_blocks * job.n_splits;
    if (blocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(deposit_kernel<true>, dim3((unsigned)blocks), dim3(kCellsPerBlock), 0, s,
                       job);
    return hipGetLastError();
}

hipError_t launch_readout(const double* acc, int64_t n_c, int64_t n_t, bool mixed, double* E,
                          double* B, hipStream_t s)
{
    if (n_c <= 0)
        return hipSuccess;
    if (mixed)
        hipLaunchKernelGGL(readout_kernel<true>, dim3((unsigned)n_c), dim3(256), 0, s, acc, n_t, E,
                           B);
    else
        hipLaunchKernelGGL(readout_kernel<false>, dim3((unsigned)n_c), dim3(256), 0, s, acc, n_t, E,
                           B);
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

}  // namespace radio
