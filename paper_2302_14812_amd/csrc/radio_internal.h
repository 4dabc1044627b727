// Internal declarations shared by the host runtime and the kernel file of libradio.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace radio {

// One trajectory state as the deposit reads it, laid out per arithmetic mode
// (the states of one particle are contiguous): position, beta, 1/gamma^2 and
// betadot = (beta_s - beta_{s-1})/dt (zero for the first state of a chunk,
// which carries no segment).  The mixed modes keep position and beta, which
// enter the arrival time and n - beta, in double, and the particle's
// (q/c) betadot and 1/(2 gamma^2), the forms their field uses, in single
// precision.  Records are 80 (double) and 64 (mixed) bytes, multiples
// of 16 so that staging copies and LDS reads stay 16-byte aligned.
struct RecF64 {
    double x[3];
    double b[3];
    double bd[3];
    double g2i;
};
struct RecMix {
    double x[3];
    double b[3];
    float bdq[3];  // (q/c) betadot of the state's particle
    float g2ih;    // 1/(2 gamma^2)
};
static_assert(sizeof(RecF64) == 80 && sizeof(RecMix) == 64, "state record layouts");

// arithmetic of a deposit: field in double, accumulation in double; field in
// single, accumulation in double; field in single, accumulation in compensated
// single pairs in HBM (the on-chip slot ring sums in double in every mode)
constexpr int kModeF64 = 0;
constexpr int kModeMix = 1;
constexpr int kModeMixTwoSum = 2;

inline size_t rec_bytes(int mode)
{
    return mode == kModeF64 ? sizeof(RecF64) : sizeof(RecMix);
}

// Workgroup shapes of the deposit: 256 threads, a tile of `cells` detector cells,
// 256 / cells particle lanes per cell (the particles of one staged batch), runs of
// `run` segments.  Shape 0 is the default; the others are compiled for the
// default detector options only, and the autotuner picks among them.
constexpr int kDepositThreads = 256;
struct TileShape {
    int cells;  // cells per tile
    int run;    // segments per run
};
constexpr int kShapes = 3;
constexpr TileShape kShapeTable[kShapes] = {{16, 16}, {8, 16}, {16, 8}};
constexpr int shape_cells(int s) { return kShapeTable[s].cells; }
constexpr int shape_groups(int s) { return kDepositThreads / kShapeTable[s].cells; }
constexpr int shape_run(int s) { return kShapeTable[s].run; }
constexpr bool shapes_valid()
{
    for (int s = 0; s < kShapes; ++s) {
        const int c = shape_cells(s), g = shape_groups(s);
        if (c * g != kDepositThreads || (g & (g - 1)) != 0 || (c & (c - 1)) != 0 || g < 4 ||
            g > 32 || shape_run(s) % 8 != 0)
            return false;
    }
    return true;
}
static_assert(shapes_valid(), "tile shapes");
// the default shape's constants (shape 0)
constexpr int kTileCells = shape_cells(0);
constexpr int kGroups = shape_groups(0);
constexpr int kRunL = shape_run(0);
constexpr int kMaxGroups = 32;                          // particles per batch, any shape
constexpr int kRingMargin = 2;                          // ring slots kept below a batch's start
constexpr int kXcds = 8;                                // accelerator dies sharing one L2 each
constexpr int kCounters = 4;  // a detector's device counters (DepositJob::counters)

// Slots per cell in the LDS ring (the small one a power of two), 48 B per slot in every mode
// (6 doubles, or 6 compensated single pairs).  Each tile takes the small ring
// when the slots a batch touches fit it (four workgroups per CU), else the
// large one (two per CU): slowly advancing arrivals, where many segments
// share a slot, fit the small ring; arrivals that cross a slot every segment
// or two need the large one.
#ifndef RADIO_RING_SMALL
#define RADIO_RING_SMALL 16
#endif
#ifndef RADIO_RING_LARGE
#define RADIO_RING_LARGE 64
#endif
// segments a large-ring workgroup stages at most per batch (longer runs are
// staged in parts of this length): what the large ring's span allows
#ifndef RADIO_LARGE_STAGE
#define RADIO_LARGE_STAGE 16
#endif
constexpr int kRingSmall = RADIO_RING_SMALL;
constexpr int kRingLarge = RADIO_RING_LARGE;
constexpr int kLargeStage = RADIO_LARGE_STAGE;

// One (detector, chunk) deposit as the kernels see it.  Sizes are 64-bit; the
// host runtime has validated every pointer and size before filling this in.
struct DepositJob {
    const double* cells;            // [n_c][3], internal (tile-ordered) rows
    double* acc;                    // [n_c][n_t][6] doubles, or [n_c][n_t][12] floats (hi, lo)
                                    // for the compensated single mode
    unsigned long long* counters;   // [kCounters]: clipped, nonmonotone, ring bypasses,
                                    // interactions deposited through the large ring
    const double* x;                // state 0 of [3][...][n_p] (components xs_stride apart)
    const double* u;                // the same for u
    const double* q;                // [n_p] or nullptr (all -1)
    void* recs;                     // workspace [n_p][n_s+1] records of the job's mode
    int32_t* perm;                  // workspace [n_groups][n_tiles][n_p]: particle orders
    uint8_t* ring_sel;              // workspace [n_tiles]: 1 where a tile takes the large ring
    const double* far;              // far-field detector: [n_c][4] n_cell, R_cell; else nullptr
    double vscale;                  // 1, or 0 for an acceleration-only detector
    int64_t hold;                   // field a segment holds: 0 current, 1 previous, 2 linear
    int64_t potentials;             // 1: deposit the potentials (A, phi) instead of (E, B)
    int64_t n_c, n_t, n_p, n_s;
    double t_first, dt;             // state s at t_first + (s0 + s)*dt
    int64_t s0;                     // the chunk's first state within its run
    int64_t xs_stride;              // elements between the components of x and u
    int64_t s_before, s_after;      // states x and u hold before state 0 and after state n_s
                                    // (a time slice of a longer chunk: its neighbours)
    double t0, inv_dt_det;          // slot coordinate (t_det - t0) / dt_det, inv_dt_det =
                                    // RN(1/dt_det)
    double dt_det;
    int64_t slot_div;               // 1: the double slot coordinate divides (the divisor
                                    // fails the check of slot_quotient_corrects)
    double inv_c, c;
    // workgroup shape (kShapeTable): its index, cells per tile, particles per batch
    // (groups) and segments per run
    int32_t shape, tile_cells, groups, run_l;
    // work decomposition, filled by plan_job()
    int64_t n_tiles;                // tiles of tile_cells cells
    int64_t n_runs;                 // runs of run_l segments
    int64_t runs_per_split;         // runs per work item
    int64_t n_splits;               // run ranges per tile
    int64_t batches_per_part;       // batches of `groups` particles per work item
    int64_t n_parts;                // particle ranges per tile and run range
    int64_t runs_per_group;         // runs sharing one particle order per tile (a power of 2)
    int64_t group_shift;            // log2(runs_per_group)
    int64_t n_groups;               // particle orders per tile
};

// One unit of a batched deposit: a tile of cells against a range of runs of one job.
struct WorkItem {
    int32_t job;
    int32_t tile;
    int32_t split;
    int32_t part;
};

// Work items are kept short (a run, or the few runs that make at least this
// many batches of particles): workgroups running at the same time then
// stream the records of few runs, which stay in cache for the many tiles that
// read them.
constexpr int64_t kMinItemBatches = 64;

// Set the job's workgroup shape (its tile, batch and run sizes).
void set_shape(DepositJob& job, int shape);
// Split the runs of a job into work items: until tiles x splits reaches
// target_blocks when it is positive, else into short items (a run or a few)
// while at least `capacity` items (the workgroups resident at once) remain;
// with fewer than two rounds of items, also into ranges of the tile's sorted
// particles (parts of at least 16 batches).
void plan_job(DepositJob& job, int target_blocks, int64_t capacity);
// the tile's sorted batches in `parts` contiguous ranges (1: all of them)
void set_parts(DepositJob& job, int64_t parts);
// One particle order per tile for each group of runs (sorted at the group's
// middle state): arrival offsets that drift apart over a long chunk are
// re-sorted along it.  max_order_groups is how many orders fit the budget
// (budget_mib, or when 0 the size of the chunk's state records and at least
// 1 GiB); set_groups spreads the job's runs over at most that many groups.
// Chunks of fewer than 16 batches of particles keep one order.
int64_t max_order_groups(const DepositJob& job, size_t rec_bytes, int64_t budget_mib);
void set_groups(DepositJob& job, int64_t max_groups);
// Runs per order group that a deposit keeps to, by depositing a longer chunk
// in time slices whose orders fit the budget; particles below which a chunk
// keeps a single order (16 batches of the job's shape).
constexpr int64_t kRunsPerGroup = 2;
inline int64_t min_group_particles(const DepositJob& job)
{
    return 16 * (int64_t)job.groups;
}

hipError_t launch_zero(double* p, int64_t n, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s);
hipError_t launch_kinematics(const DepositJob& job, int mode, hipStream_t s);
hipError_t launch_order(const DepositJob& job, hipStream_t s);
hipError_t launch_ring_choice(const DepositJob& job, int mode, hipStream_t s);
hipError_t launch_deposit(const DepositJob& job, int mode, int64_t max_grid, hipStream_t s);
// Deposit kernel variants: for shape 0, v = mode + 3 * (G + 4 * hold) with
// G = far + 2 * potentials (36); for the other shapes, the default options only:
// v = 36 + 3 * (shape - 1) + mode.
constexpr int kOptionVariants = 36;
constexpr int kKernelVariants = kOptionVariants + 3 * (kShapes - 1);
inline int kernel_variant(int mode, const DepositJob& J)
{
    const int G = (J.far ? 1 : 0) + (J.potentials ? 2 : 0);
    if (J.shape != 0)
        return (G == 0 && J.hold == 0) ? kOptionVariants + 3 * (J.shape - 1) + mode : -1;
    return mode + 3 * (G + 4 * (int)J.hold);
}
// next: two work counters (small-ring and large-ring workgroups)
hipError_t launch_deposit_batch(const DepositJob* jobs, const WorkItem* items, int64_t n_items,
                                unsigned long long* next, int variant, int blocks_small,
                                int blocks_large, hipStream_t s);
int persistent_blocks_per_cu(int variant, bool large_ring);
hipError_t launch_readout(const double* acc, int64_t n_c, int64_t n_t, const int64_t* user_index,
                          bool pairs, double* E, double* B, hipStream_t s);
// E and B [n_c][n_t][3] in the caller's cell order into the accumulator (the
// inverse of launch_readout)
hipError_t launch_load(double* acc, int64_t n_c, int64_t n_t, const int64_t* user_index,
                       bool pairs, const double* E, const double* B, hipStream_t s);
// spectral post-processing (radio_spectrum.hip): one group of G cells (internal
// rows r0 ..) through load, FFT passes and power; work0/work1 hold 2 G N values,
// tables kSpecTableValues (twiddle tables, rewritten by each call).  Where the
// transform reads the detector in a way that allows it, the group's dI/dOmega
// is computed on the way (dIdO set) and *parseval_done says so.
constexpr int64_t kSpecTableValues = 5120;
hipError_t launch_spectrum_group(const double* acc, bool pairs, int64_t n_t, int64_t r0,
                                 int64_t G, int64_t N, const double* cells,
                                 const int64_t* user_index, const double* weights, double dt,
                                 double c, double2* work0, double2* work1, double2* tables,
                                 double* d2I, double* dIdw, double* dIdO, bool* parseval_done,
                                 bool first_group, hipStream_t s);
hipError_t launch_spectrum_parseval(const double* acc, bool pairs, int64_t n_c, int64_t n_t,
                                    const double* cells, const int64_t* user_index, double dt,
                                    double c, double* dIdO, hipStream_t s);
// the run-time push (radio_push.hip)
struct PushParams {
    double qm, dt;
    double E[3], B[3];
    double wave_amplitude;
    double wave_dir[3], wave_pol[3];
    double wave_omega, wave_phase;
};
hipError_t launch_push(const PushParams& P, int64_t n_p, int64_t n_s, double t_first,
                       int64_t first_step, double* x, double* u, hipStream_t s);
hipError_t launch_arrival(const double* cells, const double* pts, const double* t, int64_t n,
                          double inv_c, double* out, hipStream_t s);
hipError_t launch_slot_coords(const double* cells, const double* pts, const double* t, int64_t n,
                              double inv_c, double t0, double dt_det, double inv_dt_det,
                              bool slot_div, double* out, hipStream_t s);
// Whether the double deposit's slot coordinate, (t_det - t0) / dt_det formed from
// RN(1/dt_det) with two corrections, is correctly rounded for every numerator
// with this divisor (|b RN(1/b) - 1| B < 1 - 2^-45, B the significand of b as
// an integer); if not, the kernels divide.
bool slot_quotient_corrects(double dt_det);

}  // namespace radio
