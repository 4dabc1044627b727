// Internal declarations shared by the host runtime and the kernel file of libradio.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace radio {

// One (detector, chunk) deposit as the kernels see it.  Sizes are 64-bit; the
// host runtime has validated every pointer and size before filling this in.
struct DepositJob {
    const double* cells;            // [n_c][3]
    double* acc;                    // [n_c][n_t][6] doubles, or [n_c][n_t][12] floats (hi, lo)
    unsigned long long* counters;   // [2]: clipped, nonmonotone
    const double* x;                // [3][n_s+1][n_p]
    const double* u;                // [3][n_s+1][n_p]
    const double* q;                // [n_p] or nullptr (all -1)
    int64_t n_c, n_t, n_p, n_s;
    double t_first, dt;             // state s at t_first + s*dt
    double t0, inv_dt_det;          // slot coordinate (t_det - t0) * inv_dt_det
    double inv_c, c;
    // work decomposition, filled by plan_job()
    int64_t n_pb;                   // particle blocks of kTileP
    int64_t n_tiles;                // runs * particle blocks
    int64_t tiles_per_split;        // tiles per workgroup along grid.y
    int64_t n_splits;
    int64_t cell_blocks;            // workgroups along the cells
};

// tile shape of the deposit kernels
constexpr int kCellsPerBlock = 256;  // one cell per lane, 4 waves
constexpr int kTileP = 16;           // particles staged per tile
constexpr int kRunL = 32;            // segments per run (states kRunL + 1)

void plan_job(DepositJob& job, int target_blocks);

hipError_t launch_zero(double* p, int64_t n, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s);
hipError_t launch_deposit_fp64(const DepositJob& job, hipStream_t s);
hipError_t launch_deposit_mixed(const DepositJob& job, hipStream_t s);
hipError_t launch_readout(const double* acc, int64_t n_c, int64_t n_t, bool mixed, double* E,
                          double* B, hipStream_t s);
hipError_t launch_arrival(const double* cells, const double* pts, const double* t, int64_t n,
                          double inv_c, double* out, hipStream_t s);

}  // namespace radio
