/*
 * radio.h -- C interface of the MI355X radiation-deposit library (libradio.so).
 *
 * The library computes the spatiotemporal radiation of charged-particle
 * trajectories the way RaDiO does (Pardal et al., "RaDiO: an efficient
 * spatiotemporal radiation diagnostic for particle-in-cell codes"):
 * for every (particle, trajectory segment, detector cell) triple it
 * evaluates the Lienard-Wiechert fields E and B = n x E (Eq. 1) with the
 * segment's current state, maps the segment's two end states to detector
 * arrival times t_det = t + |x_cell - x_part|/c (Eq. 2, Alg. 1), and
 * deposits the field, held constant between those two arrival times, into
 * the detector's uniform time slots with the integrator-detector weights of
 * Sec. 3.2 / Alg. 2: slot j = [t0 + j dt_det, t0 + (j+1) dt_det) receives
 * the integral of the held field over the slot divided by dt_det.  Parts of
 * a segment outside the time array are dropped.
 *
 * Units follow the paper's normalised Gaussian units: c is a parameter
 * (1 in normalised units), charges are signed multiples of e, momenta are
 * u = p/(m c) = gamma beta, and fields come out in charge/length^2.
 *
 * Every call returns RADIO_OK (0) or a negative status; no call aborts or
 * throws across this interface.  On an argument error nothing is modified.
 * Work is enqueued asynchronously on the caller's HIP stream (`stream` is a
 * hipStream_t; NULL selects the null stream); the caller keeps device inputs
 * alive until the stream has passed the call.  All device pointers must
 * point to memory of the device that was current when the detector was
 * created.  Calls on one detector must be ordered by the caller (one stream,
 * or events between streams).
 */
#ifndef RADIO_H
#define RADIO_H

#include <stdint.h>

#if defined(__GNUC__)
#define RADIO_API __attribute__((visibility("default")))
#else
#define RADIO_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define RADIO_OK 0
#define RADIO_EINVAL (-1)  /* invalid argument */
#define RADIO_ENOMEM (-2)  /* device or host allocation failed */
#define RADIO_EDEVICE (-3) /* a HIP call or kernel launch failed */
#define RADIO_ESTATE (-4)  /* object in the wrong state (e.g. wrong device) */
#define RADIO_ETOOBIG (-5) /* a chunk needs more than the fixed scratch of
                              radio_deposit_trajectory_chunk_noalloc */

/* arithmetic of the deposit */
#define RADIO_FP64 0         /* every step in IEEE double */
#define RADIO_MIXED 1        /* arrival time, slot coordinate and n - beta in double;
                                kappa (a sum of positive terms), the rest of the field
                                and the slot weights in single; slot accumulation in
                                double */
#define RADIO_MIXED_TWOSUM 2 /* as RADIO_MIXED, but the detector's slots in device
                                memory are (hi, lo) single-precision pairs: every add
                                to them carries its exact rounding error (two-sum) into
                                lo; the on-chip sums that reach them are formed in
                                double */

/* detector options (bit flags in radio_detector_desc.options) */
#define RADIO_FAR_FIELD 1  /* far-field arrival time, Eq. 3: t + R_cell/c - x_part . n_cell/c
                              with R_cell = |x_cell| and n_cell = x_cell / R_cell (distance
                              and direction from the origin), and the same geometry in
                              Eq. 1 (n = n_cell, R = R_cell): no square root per
                              interaction.  Valid when the particles stay near the origin
                              compared with R_cell */
#define RADIO_ACCEL_ONLY 2 /* only the acceleration (second) term of Eq. 1, enough when
                              R gamma^2 |betadot| / c >> 1 (Sec. 2) */
#define RADIO_HOLD_PREVIOUS 4 /* segment s holds the field of state s-1 (the Fig. 5
                                 walk-through) instead of that of state s (Alg. 1, the
                                 default); a chunk's first state takes the forward
                                 difference for betadot */
#define RADIO_HOLD_LINEAR 8   /* the field varies linearly in arrival time from E_{s-1} to
                                 E_s, each with betadot centred at its state (one-sided at
                                 the chunk's ends): the higher-order interpolation named as
                                 an extension in Sec. 6.  Excludes RADIO_HOLD_PREVIOUS */
#define RADIO_POTENTIALS 16   /* the Lienard-Wiechert potentials phi = q/(kappa R) and
                                 A = q beta/(kappa R) instead of the fields (the extension
                                 named in Sec. 6), deposited with the same hold rule and
                                 weights; radio_read_detector then returns A in E's place
                                 and (phi, 0, 0) in B's.  Excludes RADIO_ACCEL_ONLY */

/* detector cell geometry (Sec. 3.1: spherical grids centred at the origin and
   cartesian planes) */
#define RADIO_GEOM_EXPLICIT 0 /* cells[n_cells][3] given by the caller */
#define RADIO_GEOM_PLANE 1    /* n1 x n2 cell centres origin + a1 e1 + a2 e2,
                                 a_i = -half_i + (i + 1/2) 2 half_i / n_i */
#define RADIO_GEOM_SPHERE 2   /* n1 x n2 cells on a sphere of `radius` about the origin:
                                 longitude (about axis x e1) and latitude measured from
                                 `axis`, spanning +-half1 and +-half2 radians, cell centres
                                 at bin middles: radius*(cos(lat)(cos(lon) axis +
                                 sin(lon) e1') + sin(lat) e2'), e1' = e1 made orthogonal
                                 to axis and normalised, e2' = axis x e1' */

typedef struct radio_detector radio_detector; /* opaque, owned by the library */

typedef struct radio_detector_desc {
    int32_t geometry;     /* RADIO_GEOM_* */
    int32_t precision;    /* RADIO_FP64, RADIO_MIXED or RADIO_MIXED_TWOSUM */
    int64_t n_cells;      /* EXPLICIT only: number of cells */
    const double* cells;  /* EXPLICIT only: HOST pointer to [n_cells][3] positions; copied */
    double origin[3];     /* PLANE: grid centre */
    double axis[3];       /* SPHERE: direction of the grid centre (need not be unit) */
    double e1[3];         /* PLANE: first grid axis; SPHERE: longitude direction */
    double e2[3];         /* PLANE: second grid axis */
    double radius;        /* SPHERE: radius */
    int64_t n1, n2;       /* PLANE/SPHERE: cells along e1 and e2; cell index = i2*n1 + i1 */
    double half1, half2;  /* PLANE: half spans; SPHERE: half apertures in radians */
    double t0;            /* start of the detector time array */
    double dt_det;        /* slot width, > 0 */
    int64_t n_t;          /* number of slots, >= 1 */
    double c;             /* speed of light, > 0 (1 in normalised units) */
    int32_t options;      /* RADIO_FAR_FIELD | RADIO_ACCEL_ONLY | RADIO_HOLD_* |
                             RADIO_POTENTIALS, or 0 (Eq. 2, all of Eq. 1, the current state's
                             field held) */
    int64_t n3;           /* SPHERE: concentric shells (0 or 1: one) of radii radius +
                             k radius_step, k < n3 (Sec. 3.1: spherical grids of several
                             radii about the origin); cell index = (k n2 + i2) n1 + i1.
                             Other geometries: 0 or 1 */
    double radius_step;   /* SPHERE: radial spacing of the shells */
} radio_detector_desc;

/*
 * A chunk of trajectory: n_steps + 1 states of n_particles particles.  State s
 * of the chunk is state first_step + s of its run, at time
 * t_first + (first_step + s)*dt (time step n of a run sits at n*dt, Sec. 3.1),
 * so a chunk cut out of a longer one keeps the exact state times of the
 * whole.  Segment s (1..n_steps) joins states s-1 and s and
 * carries the field of state s (beta_s, betadot_s = (beta_s - beta_{s-1})/dt),
 * as Alg. 1 passes the current step's E(n, beta, betadot) to the deposit.
 * Streaming: consecutive chunks share one state (state 0 of a chunk is the
 * last state of the previous one), which makes deposits stateless, additive
 * and order independent.
 */
typedef struct radio_chunk {
    int64_t n_particles;  /* >= 0 (0 deposits nothing) */
    int64_t n_steps;      /* segments, >= 0 (0 deposits nothing) */
    double t_first;       /* time of the run's state 0 */
    double dt;            /* time between states, > 0 */
    int64_t first_step;   /* index in its run of the chunk's state 0, >= 0;
                             first_step + n_steps < 2^53 */
    const double* x;      /* DEVICE [3][n_steps+1][n_particles] positions (SoA) */
    const double* u;      /* DEVICE [3][n_steps+1][n_particles] momenta p/(m c) */
    const double* q;      /* DEVICE [n_particles] signed charges, or NULL for all -1 */
} radio_chunk;

typedef struct radio_stats {
    int64_t interactions; /* (particle segment, cell) pairs deposited so far */
    int64_t clipped;      /* of those, pairs with some part outside the time array */
    int64_t nonmonotone;  /* of those, pairs whose arrival time decreases (|dx| > c dt) */
    int64_t chunks;       /* deposit calls accepted */
    int64_t bytes;        /* device bytes held by the detector (with its workspace) */
    int64_t bypassed;     /* slot updates that missed the on-chip slot window and went
                             straight to device memory (a performance counter) */
    int64_t slices;       /* deposit launches made for those chunks: a long chunk runs
                             as time slices (radio_tuning), alone or in a batch; any
                             other batched chunk as one job of the batch's launch */
    int64_t large_ring;   /* of the interactions, those deposited by tiles that took the
                             large on-chip slot ring (arrivals crossing slots often; a
                             performance counter) */
} radio_stats;

/*
 * Create a detector on the current device: copies the cell positions, allocates
 * and zeroes the slot accumulator (n_cells * n_t * 6 doubles) with work
 * enqueued on `stream`.  *out receives the handle.  RADIO_EINVAL for a bad
 * description, RADIO_ENOMEM if the accumulator does not fit.
 */
RADIO_API int radio_detector_create(const radio_detector_desc* desc, void* stream, radio_detector** out);

/* Wait for the device, then free everything the detector holds.  NULL is a no-op. */
RADIO_API int radio_detector_destroy(radio_detector* det);

/* Zero the accumulated fields and statistics (enqueued on `stream`). */
RADIO_API int radio_detector_reset(radio_detector* det, void* stream);

/*
 * Deposit one chunk (Alg. 1 over every particle, cell and segment; Alg. 2 for
 * each).  Validates the chunk on the host; RADIO_EINVAL (nothing enqueued) for
 * NULL pointers with a nonempty chunk, dt <= 0, non-finite times or negative
 * sizes.  Input values are not inspected: NaN positions or momenta give NaN or
 * dropped deposits, never out-of-bounds writes.
 */
RADIO_API int radio_deposit_trajectory_chunk(radio_detector* det, const radio_chunk* chunk, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the deposit
 * of radio_deposit_trajectory_chunk, same arguments and result up to the order
 * of floating-point additions, with every workspace in one fixed device array
 * of radio_noalloc_scratch_bytes() bytes (256 MiB) per GPU, held by the
 * library from its first use on that GPU until the process ends.  It calls no
 * allocation or release routine.  The chunk runs as time slices of whole runs
 * sized so that a slice's state records, particle orders (one per two runs of
 * 16 segments: 4 * ceil(n_cells / 16) * n_particles bytes each) and ring choices
 * fit the array; RADIO_ETOOBIG (nothing enqueued) when even one run does not.
 * All calls on one GPU share the array: calls on one stream follow each other,
 * calls that overlap on one GPU from different streams race and must not be
 * made.  Argument checks and other errors as radio_deposit_trajectory_chunk.
 */
RADIO_API int radio_deposit_trajectory_chunk_noalloc(radio_detector* det, const radio_chunk* chunk,
                                                     void* stream);

/* The size of the non-allocating deposit's scratch per GPU, in bytes. */
RADIO_API int radio_noalloc_scratch_bytes(int64_t* bytes);

/*
 * Deposit n independent (detector, chunk) pairs in one persistent launch per
 * precision present: the pairs' work is cut into items (a tile of cells x a
 * range of runs), ordered longest first, and taken by resident workgroups
 * from a device counter.  The result equals n separate
 * radio_deposit_trajectory_chunk calls (up to the order of floating-point
 * additions).  A pair whose particle orders would not fit the order budget
 * (radio_tuning) is deposited after the persistent launch, in the time slices
 * of a single deposit.  All detectors must live on the current device; a
 * detector may appear more than once.  On any invalid pair nothing is
 * enqueued; RADIO_ENOMEM leaves every detector unchanged.  Batch
 * workspaces are shared by the device's batches, two in turn: a call waits
 * (on the host) for the batch enqueued two calls earlier on that device to
 * finish, so one batch can run while the next is prepared.
 */
RADIO_API int radio_deposit_batch(radio_detector* const* dets, const radio_chunk* chunks, int n,
                        void* stream);

/*
 * Launch tunables, process wide (the autotuner sets them):
 *   target_blocks        workgroups aimed at by a single deposit (the runs of a
 *                        chunk are split until tiles x splits reaches it); 0, the
 *                        default, splits into short items of one run or a few
 *   max_grid             workgroups of one launch of a single deposit (1 ..
 *                        2^22, the default): more work items run as several
 *                        launches
 *   items_per_workgroup  work items per resident workgroup in a batched deposit
 *                        (finer items balance uneven jobs, coarser ones cost less)
 *   order_budget_mib     device memory (MiB) the per-tile particle orders of one
 *                        deposit may take; 0, the default, allows the size of the
 *                        chunk's state records and at least 1 GiB.  A single
 *                        deposit, alone or batched, keeps each order to at most
 *                        two runs (arrival offsets drift apart along a chunk);
 *                        a chunk whose orders exceed the budget is deposited in
 *                        time slices that fit it, with the same result up to
 *                        summation order
 *   shape                workgroup shape of the deposit of detectors with the
 *                        default options (0 for the others): 0 = tiles of 16
 *                        cells against batches of 16 particles and runs of 16
 *                        segments (the default), 1 = 8 cells x 32 particles x
 *                        16 segments, 2 = 16 cells x 16 particles x 8 segments.
 *                        Every shape gives the same result up to summation
 *                        order; the autotuner picks the fastest per workload
 */
typedef struct radio_tuning {
    int32_t target_blocks;
    int32_t items_per_workgroup;
    int32_t max_grid;
    int32_t order_budget_mib;
    int32_t shape;
} radio_tuning;

RADIO_API int radio_set_tuning(const radio_tuning* t);
RADIO_API int radio_get_tuning(radio_tuning* t);

/*
 * Write the detector fields: E and B as DEVICE arrays [n_cells][n_t][3]
 * (double), slot values as defined above.  Either pointer may be NULL to skip
 * it.  Does not modify the detector.
 */
RADIO_API int radio_read_detector(const radio_detector* det, double* E, double* B, void* stream);

/*
 * Replace the detector's fields with E and B, DEVICE arrays [n_cells][n_t][3]
 * (double) in the layout radio_read_detector writes: the inverse of a read, so
 * that a snapshot read from a detector and loaded into a detector of the same
 * description (cells, t0, dt_det, n_t, precision, options) resumes its
 * accumulation -- a checkpoint.  The slot array is the detector's only state
 * (the integrator detector of Sec. 3.2; chunks carry their previous state,
 * Sec. 3.1), so later deposits add to the loaded fields as they would have to
 * the original ones.  Exact for RADIO_FP64 and RADIO_MIXED; RADIO_MIXED_TWOSUM
 * stores each value as a (hi, lo) single-precision pair, to about 2^-48 of it.
 * Statistics (radio_detector_stats) are not changed.  Both pointers are
 * required (RADIO_EINVAL otherwise); the arrays are read by work enqueued on
 * `stream` and must stay valid until it has run.
 */
RADIO_API int radio_detector_load(radio_detector* det, const double* E, const double* B,
                                  void* stream);

/* Statistics; synchronises the device to read the counters. */
RADIO_API int radio_detector_stats(const radio_detector* det, radio_stats* out);

/* Shape of a detector: cells, slots, precision (any pointer may be NULL). */
RADIO_API int radio_detector_shape(const radio_detector* det, int64_t* n_cells, int64_t* n_t,
                         int32_t* precision);

/* Copy the detector's cell positions to HOST memory out[n_cells][3]. */
RADIO_API int radio_detector_cells(const radio_detector* det, double* out);

/*
 * External fields of the run-time push: uniform E and B plus an optional plane
 * wave E_w = wave_amplitude * wave_pol * cos(wave_omega (t - wave_dir . x) +
 * wave_phase), B_w = wave_dir x E_w (c = 1; wave_dir and wave_pol unit and
 * perpendicular).
 */
typedef struct radio_push_desc {
    double qm;              /* charge-to-mass ratio in the units of E and B (-1: electrons) */
    double dt;              /* time step, > 0 */
    double E[3];
    double B[3];
    double wave_amplitude;  /* 0: no wave */
    double wave_dir[3];
    double wave_pol[3];
    double wave_omega;
    double wave_phase;
} radio_push_desc;

/*
 * The particle push of the run-time mode (Sec. 3.1: the deposit is a sub-step
 * right after each push, reading the new and the stored states).  Boris method
 * with x and u kept as samples at the same times: half drift, Boris kick with
 * the fields at the half step, half drift.  x and u are DEVICE arrays
 * [3][n_steps+1][n_particles] (the chunk layout of radio_chunk); state 0 is
 * read, states 1..n_steps are written.  State s is at t_first +
 * (first_step + s) dt, so the arrays then form a chunk that
 * radio_deposit_trajectory_chunk (or radio_deposit_batch) takes as it is, with
 * no copy through the host.  Asynchronous on `stream`.  RADIO_EINVAL for a
 * NULL or invalid argument.
 */
RADIO_API int radio_push(const radio_push_desc* d, int64_t n_particles, int64_t n_steps,
                         double t_first, int64_t first_step, double* x, double* u, void* stream);

/*
 * Spectral post-processing (Sec. 4: the detector data Fourier transformed with
 * respect to time, the route by which the paper checks its deposit against the
 * spectra of Eq. 7 and Eq. 8).  A slot holds the field averaged over the slot,
 * so the transform of the piecewise-constant signal of cell c is
 *     F_c(omega) = sum_j E_cj e^{-i omega j dt_det} (e^{-i omega dt_det} - 1)/(-i omega)
 * and, with R_c = |x_c| the cell's distance from the origin,
 *     d2I[c][m] = c R_c^2 / (4 pi^2) |F_c(omega_m)|^2     (d2I/domega dOmega)
 *     dIdw[m]   = sum_c weight_c d2I[c][m]                 (dI/domega)
 *     dIdO[c]   = c R_c^2 / (4 pi) sum_j |E_cj|^2 dt_det   (dI/dOmega, Parseval)
 * at omega_m = 2 pi m / (n_fft dt_det), m = 0 .. n_fft/2, the signal zero
 * beyond its n_t slots.  In double precision for every detector precision.
 *   n_fft   a power of two >= n_t, <= 2^30; 0 picks the smallest one
 *   weights HOST [n_cells] per-cell weights of dIdw in the caller's cell order
 *           (e.g. solid angles), or NULL for 1
 *   d2I     DEVICE [n_cells][n_fft/2 + 1] in the caller's cell order, or NULL
 *   dIdw    DEVICE [n_fft/2 + 1], or NULL
 *   dIdO    DEVICE [n_cells] in the caller's cell order, or NULL
 * Work is enqueued on `stream`, after the deposits already there, and the call
 * waits for the stream before returning.  The detector keeps the workspace of
 * d2I and dIdw (two complex arrays per group of cells: about 1 GiB, or
 * 64 n_fft bytes when one cell needs more) for later spectra;
 * radio_detector_destroy releases it.  RADIO_EINVAL for a bad n_fft or
 * no output, RADIO_ENOMEM if the workspace cannot be had.
 */
RADIO_API int radio_spectrum(radio_detector* det, int64_t n_fft, const double* weights,
                             double* d2I, double* dIdw, double* dIdO, void* stream);

/*
 * Arrival times t + |x_cell - x|/c (Eq. 2) of n explicit (cell, point, time)
 * triples, evaluated on the device with exactly the rounding the deposit uses:
 * t_s = t_first + s*dt is the caller's job; here t is given.  DEVICE arrays:
 * cells[n][3], points[n][3], t[n], out[n].
 */
RADIO_API int radio_arrival_times(const double* cells, const double* points, const double* t, int64_t n,
                        double c, double* out, void* stream);

/*
 * Slot coordinates (t + |x_cell - x|/c - t0) / dt_det of n explicit (cell,
 * point, time) triples: the arrival time of Eq. 2 in units of slots from the
 * start of a time array (t0, dt_det), whose integer part is the slot Alg. 2
 * deposits into.  Evaluated on the device with exactly the rounding of the
 * double-precision deposit: the arrival time as radio_arrival_times, then the
 * correctly rounded quotient.  DEVICE arrays cells[n][3], points[n][3], t[n],
 * out[n].  RADIO_EINVAL for c or dt_det not positive and finite (or 1/dt_det
 * not finite), t0 not finite, or a NULL array with n > 0.
 */
RADIO_API int radio_slot_coordinates(const double* cells, const double* points, const double* t,
                                     int64_t n, double c, double t0, double dt_det, double* out,
                                     void* stream);

/* Human-readable text for a status code (static storage). */
RADIO_API const char* radio_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* RADIO_H */
