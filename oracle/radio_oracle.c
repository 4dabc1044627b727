/*
 * radio_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU implementation of the RaDiO radiation
 * deposit (Pardal et al., "RaDiO: an efficient spatiotemporal radiation
 * diagnostic for particle-in-cell codes").  It exists to check the GPU
 * library and is only ever called by the tests, by the package's smoke
 * check and by the CPU-baseline leg of the benchmark.  It shares no code,
 * header or constant with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math), so
 * every + - * / sqrt below is one IEEE double operation rounded to nearest.
 *
 * What it computes (per detector cell c, particle p, segment s = 1..S):
 *   kinematics (Alg. 1, velocity and acceleration lines):
 *       g      = |u_s|^2 + 1,   beta_s = u_s / sqrt(g),   1/gamma_s^2 = 1/g
 *       betadot_s = (beta_s - beta_{s-1}) / dt
 *   arrival time (Eq. 2, Alg. 1):  tau_s = t_s + |x_c - x_{p,s}| / c,
 *       t_s = t_first + (first_step + s)*dt   (state s of a chunk is the run's
 *       state first_step + s; time step n of the run sits at n*dt, Sec. 3.1)
 *   Lienard-Wiechert field of the segment (Eq. 1), with the current state's
 *   quantities (Alg. 1 passes E(n, beta, betadot) of the current step):
 *       n = (x_c - x_{p,s}) / R   (from the particle towards the cell, Sec. 2)
 *       kappa = 1 - n.beta
 *       E = q (n - beta) / (gamma^2 kappa^3 R^2)
 *           + (q/c) n x ((n - beta) x betadot) / (kappa^3 R)
 *       B = n x E
 *   integrator-detector deposit (Sec. 3.2, Alg. 2): the field is held
 *   constant between the arrival times tau_{s-1} and tau_s, and slot j,
 *   [t0 + j dt_det, t0 + (j+1) dt_det), receives the integral of that
 *   piecewise-constant signal over the slot divided by dt_det:
 *       D[c][j] += (E, B) * |[lo, hi] cap slot_j| / dt_det,
 *       lo = min(tau_{s-1}, tau_s), hi = max(tau_{s-1}, tau_s).
 *   Parts outside the detector's time array are dropped.
 *
 * Canonical evaluation order (the quantities that cancel, so both
 * implementations must round them the same way; every other line may be
 * evaluated in any order):
 *   |v|^2 = (v0*v0 + v1*v1) + v2*v2 ;  g = |u|^2 + 1 ;  beta_k = u_k / sqrt(g)
 *   t_s  = t_first + (double)(first_step + s) * dt ;  R = sqrt(|x_c - x_s|^2)
 *   tau  = t_s + R * (1/c)          ;  n_k = d_k * (1/R)
 *   slot coordinate (tau - t0) / dt_det, one correctly rounded division: the
 *   time in units of slots, whose integer part is the slot of Alg. 2 (a
 *   segment much shorter than a slot changes length by ulp(coordinate)/length
 *   if rounded differently)
 *   kappa = (|n - beta|^2 + 1/g) / 2, which equals 1 - n.beta exactly for a
 *   unit n (|n - beta|^2 = 1 - 2 n.beta + |beta|^2 and 1 - |beta|^2 = 1/g)
 *   but has no cancellation as beta -> 1.
 *
 * Detector options (bit flags, may be combined):
 *   FAR_FIELD (1): the far-field arrival time of Eq. 3,
 *       tau_s = t_s + (R_cell - x_{p,s} . n_cell) / c,
 *       R_cell = |x_c|, n_cell = x_c / R_cell (the cell's distance and
 *       direction from the origin), and the field of Eq. 1 with the same
 *       far-field geometry: n = n_cell and R = R_cell.
 *       Canonical order: R_cell = sqrt(|x_c|^2), n_cell_k = x_c_k * (1/R_cell),
 *       dot = (x0*n0 + x1*n1) + x2*n2, tau = t_s + (R_cell - dot) * (1/c).
 *   ACCEL_ONLY (2): only the second (acceleration) term of Eq. 1, which the
 *       paper keeps when R gamma^2 |betadot| / c >> 1 (Sec. 2).
 *   HOLD_PREVIOUS (4): segment s holds the field of state s-1 (the reading of
 *       the Fig. 5 walk-through, "the time until the next deposition"),
 *       instead of the field of state s (Alg. 1, the default).
 *   HOLD_LINEAR (8): the field varies linearly in arrival time from E_{s-1}
 *       at tau_{s-1} to E_s at tau_s (the higher-order interpolation the
 *       paper names as an extension, Sec. 6): slot j receives the overlap
 *       times the interpolant at the overlap's midpoint.  Each state's field
 *       then takes the centred difference betadot_s = (beta_{s+1} -
 *       beta_{s-1}) / (2 dt), one-sided at the chunk's first and last state,
 *       so that both ends of a segment are evaluated at their own times.
 *   POTENTIALS (16): the Lienard-Wiechert potentials instead of the fields
 *       (the extension named in Sec. 6): phi = q / (kappa R) and
 *       A = q beta / (kappa R) at the same retarded state (Gaussian units,
 *       c = 1 in A's normalisation as in Eq. 1); the six accumulators hold
 *       (A_x, A_y, A_z, phi, 0, 0).  Excludes ACCEL_ONLY.
 *   With HOLD_PREVIOUS, the field of a chunk's first state takes
 *   betadot_0 = (beta_1 - beta_0) / dt, the only difference the chunk holds;
 *   every other state keeps the backward difference.
 *
 * Conventions: Gaussian units, c given (1 in normalised units), signed
 * charge q per particle (a NULL charge array means q = -1, electrons).
 * Positions and momenta are structure-of-arrays float64
 *   x[(k*(S+1) + s)*Np + p],  u likewise,  k = 0..2.
 * The detector array is D[(c*n_t + j)*6 + k], k = Ex, Ey, Ez, Bx, By, Bz,
 * and is accumulated into (+=).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#define EXPORT __attribute__((visibility("default")))

#define ORACLE_FAR_FIELD 1
#define ORACLE_ACCEL_ONLY 2
#define ORACLE_HOLD_PREVIOUS 4
#define ORACLE_HOLD_LINEAR 8
#define ORACLE_POTENTIALS 16

/* beta and 1/gamma^2 from the momentum u = gamma beta (Alg. 1). */
EXPORT void radio_oracle_kinematics(const double u[3], double beta[3], double* inv_gamma2)
{
    double g = ((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]) + 1.0;
    double sq = sqrt(g);
    beta[0] = u[0] / sq;
    beta[1] = u[1] / sq;
    beta[2] = u[2] / sq;
    *inv_gamma2 = 1.0 / g;
}

/* Detector arrival time of light emitted at (x_part, t) and seen at x_cell (Eq. 2). */
EXPORT double radio_oracle_arrival(const double x_cell[3], const double x_part[3], double t,
                                   double c)
{
    double d0 = x_cell[0] - x_part[0];
    double d1 = x_cell[1] - x_part[1];
    double d2 = x_cell[2] - x_part[2];
    double R = sqrt((d0 * d0 + d1 * d1) + d2 * d2);
    return t + R * (1.0 / c);
}

/* Slot coordinate of an arrival time: (tau - t0) / dt_det, the time since the
   start of the detector's time array in units of its slot width, whose integer
   part is the slot Alg. 2 deposits into (Sec. 3.2). */
EXPORT double radio_oracle_slot_of(double tau, double t0, double dt_det)
{
    return (tau - t0) / dt_det;
}

/* The cell's distance from the origin and its direction (the far-field
   geometry of Eq. 3). */
static void far_geometry(const double x_cell[3], double n[3], double* R, double* R2)
{
    double Rc2 = (x_cell[0] * x_cell[0] + x_cell[1] * x_cell[1]) + x_cell[2] * x_cell[2];
    double Rc = sqrt(Rc2);
    double ri = 1.0 / Rc;
    n[0] = x_cell[0] * ri;
    n[1] = x_cell[1] * ri;
    n[2] = x_cell[2] * ri;
    *R = Rc;
    *R2 = Rc2;
}

/* Far-field arrival time (Eq. 3): t + R_cell/c - x_part . n_cell / c. */
EXPORT double radio_oracle_arrival_far(const double x_cell[3], const double x_part[3], double t,
                                       double c)
{
    double n[3], Rc, Rc2;
    far_geometry(x_cell, n, &Rc, &Rc2);
    double dot = (x_part[0] * n[0] + x_part[1] * n[1]) + x_part[2] * n[2];
    return t + (Rc - dot) * (1.0 / c);
}

static void cross(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

/* Eq. 1 for a given direction n (unit, towards the cell), distance R and R2 = R^2. */
static void lw_field(const double n[3], double R, double R2, const double beta[3],
                     double inv_gamma2, const double betadot[3], double q, double c,
                     int accel_only, double E[3], double B[3])
{
    double w[3] = {n[0] - beta[0], n[1] - beta[1], n[2] - beta[2]};
    double kappa = 0.5 * (((w[0] * w[0] + w[1] * w[1]) + w[2] * w[2]) + inv_gamma2);
    double k3 = kappa * kappa * kappa;
    /* velocity field: q (n - beta) / (gamma^2 kappa^3 R^2) */
    double cv = accel_only ? 0.0 : q * inv_gamma2 / (k3 * R2);
    /* acceleration field: (q/c) n x ((n - beta) x betadot) / (kappa^3 R) */
    double ca = q / (c * k3 * R);
    double wxb[3], nxwxb[3];
    cross(w, betadot, wxb);
    cross(n, wxb, nxwxb);
    for (int k = 0; k < 3; ++k)
        E[k] = cv * w[k] + ca * nxwxb[k];
    cross(n, E, B);
}

/* Lienard-Wiechert E and B at x_cell from a charge q at x_part (Eq. 1), with
   the detector options above. */
EXPORT void radio_oracle_field_opts(const double x_cell[3], const double x_part[3],
                                    const double beta[3], double inv_gamma2,
                                    const double betadot[3], double q, double c, int options,
                                    double E[3], double B[3])
{
    double n[3], R, R2;
    if (options & ORACLE_FAR_FIELD) {
        far_geometry(x_cell, n, &R, &R2);
    } else {
        double d[3] = {x_cell[0] - x_part[0], x_cell[1] - x_part[1], x_cell[2] - x_part[2]};
        R2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
        R = sqrt(R2);
        double rinv = 1.0 / R;
        n[0] = d[0] * rinv;
        n[1] = d[1] * rinv;
        n[2] = d[2] * rinv;
    }
    if (options & ORACLE_POTENTIALS) {
        double w[3] = {n[0] - beta[0], n[1] - beta[1], n[2] - beta[2]};
        double kappa = 0.5 * (((w[0] * w[0] + w[1] * w[1]) + w[2] * w[2]) + inv_gamma2);
        double phi = q / (kappa * R);
        for (int k = 0; k < 3; ++k)
            E[k] = phi * beta[k];
        B[0] = phi;
        B[1] = 0.0;
        B[2] = 0.0;
        return;
    }
    lw_field(n, R, R2, beta, inv_gamma2, betadot, q, c, (options & ORACLE_ACCEL_ONLY) != 0, E,
             B);
}

/* The exact field (no options). */
EXPORT void radio_oracle_field(const double x_cell[3], const double x_part[3],
                               const double beta[3], double inv_gamma2, const double betadot[3],
                               double q, double c, double E[3], double B[3])
{
    radio_oracle_field_opts(x_cell, x_part, beta, inv_gamma2, betadot, q, c, 0, E, B);
}

/* Add F * overlap of the slot-unit interval [lo, hi] with each slot. */
static void deposit_interval(double* Dc, int64_t n_t, double lo, double hi, const double F[6])
{
    if (!(hi > 0.0) || !(lo < (double)n_t))
        return;
    int64_t j_lo = lo <= 0.0 ? 0 : (int64_t)floor(lo);
    int64_t j_hi = hi >= (double)n_t ? n_t - 1 : (int64_t)floor(hi);
    for (int64_t j = j_lo; j <= j_hi; ++j) {
        double a = lo > (double)j ? lo : (double)j;
        double b = hi < (double)(j + 1) ? hi : (double)(j + 1);
        double w = b - a;
        if (w > 0.0) {
            double* Dj = Dc + 6 * j;
            for (int k = 0; k < 6; ++k)
                Dj[k] += F[k] * w;
        }
    }
}

/* Add the linear interpolant from Fa at slot coordinate a to Fb at b, integrated
   over each slot's overlap with [min(a,b), max(a,b)]: overlap times the
   interpolant at the overlap's midpoint. */
static void deposit_interval_linear(double* Dc, int64_t n_t, double a, double b,
                                    const double Fa[6], const double Fb[6])
{
    double lo = a < b ? a : b;
    double hi = a < b ? b : a;
    if (!(hi > 0.0) || !(lo < (double)n_t) || !(hi > lo))
        return;
    int64_t j_lo = lo <= 0.0 ? 0 : (int64_t)floor(lo);
    int64_t j_hi = hi >= (double)n_t ? n_t - 1 : (int64_t)floor(hi);
    for (int64_t j = j_lo; j <= j_hi; ++j) {
        double p = lo > (double)j ? lo : (double)j;
        double q = hi < (double)(j + 1) ? hi : (double)(j + 1);
        double w = q - p;
        if (w > 0.0) {
            /* position of the midpoint, 0 at a, from differences with a (exact for the
               coordinates of one segment), so that a segment much shorter than a slot
               keeps its relative accuracy */
            double f = 0.5 * ((p - a) + (q - a)) / (b - a);
            double* Dj = Dc + 6 * j;
            for (int k = 0; k < 6; ++k)
                Dj[k] += (Fa[k] + (Fb[k] - Fa[k]) * f) * w;
        }
    }
}

static void load_state(const double* a, int64_t n_states, int64_t n_p, int64_t s, int64_t p,
                       double out[3])
{
    for (int k = 0; k < 3; ++k)
        out[k] = a[((int64_t)k * n_states + s) * n_p + p];
}

/* Centred betadot of state s, (beta_{s+1} - beta_{s-1}) / (2 dt), one-sided at the
   chunk's ends. */
static void state_betadot(const double* u, int64_t n_states, int64_t n_p, int64_t n_steps,
                          int64_t s, int64_t p, double dt, double bd[3])
{
    int64_t a = s > 0 ? s - 1 : 0;
    int64_t b = s < n_steps ? s + 1 : n_steps;
    double ua[3], ub[3], ba[3], bb[3], ga, gb;
    load_state(u, n_states, n_p, a, p, ua);
    load_state(u, n_states, n_p, b, p, ub);
    radio_oracle_kinematics(ua, ba, &ga);
    radio_oracle_kinematics(ub, bb, &gb);
    double span = (double)(b - a) * dt;
    for (int k = 0; k < 3; ++k)
        bd[k] = (bb[k] - ba[k]) / span;
}

/*
 * The whole deposit: every (cell, particle, segment) triple of one chunk of
 * S+1 states, accumulated into D.  counters (may be NULL) receives
 * [0] segments with any part outside the time array, [1] segments whose
 * arrival times decrease.  Returns 0, or -1 on invalid arguments.
 */
EXPORT int radio_oracle_deposit(const double* cells, int64_t n_cells, double t0, double dt_det,
                                int64_t n_t, double c, int64_t n_p, int64_t n_steps,
                                double t_first, int64_t first_step, double dt, const double* x,
                                const double* u, const double* q, int options, double* D,
                                int64_t* counters, int n_threads)
{
    if (n_cells < 0 || n_t < 1 || n_p < 0 || n_steps < 0 || first_step < 0 ||
        !(dt_det > 0.0) || !(c > 0.0))
        return -1;
    if (n_cells == 0 || n_p == 0 || n_steps == 0)
        return 0;
    if (!cells || !x || !u || !D || !(dt > 0.0))
        return -1;
    const int64_t n_states = n_steps + 1;
    int64_t clipped = 0, nonmono = 0;
    if (n_threads < 1)
        n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads) reduction(+ : clipped, nonmono)
    for (int64_t ic = 0; ic < n_cells; ++ic) {
        const double* xc = cells + 3 * ic;
        double* Dc = D + ic * n_t * 6;
        for (int64_t p = 0; p < n_p; ++p) {
            double qp = q ? q[p] : -1.0;
            for (int64_t s = 1; s <= n_steps; ++s) {
                double u_prev[3], u_cur[3], x_prev[3], x_cur[3];
                load_state(u, n_states, n_p, s - 1, p, u_prev);
                load_state(u, n_states, n_p, s, p, u_cur);
                load_state(x, n_states, n_p, s - 1, p, x_prev);
                load_state(x, n_states, n_p, s, p, x_cur);
                double beta_prev[3], beta[3], g2p, g2;
                radio_oracle_kinematics(u_prev, beta_prev, &g2p);
                radio_oracle_kinematics(u_cur, beta, &g2);
                double betadot[3];
                for (int k = 0; k < 3; ++k)
                    betadot[k] = (beta[k] - beta_prev[k]) / dt;
                double t_prev = t_first + (double)(first_step + s - 1) * dt;
                double t_cur = t_first + (double)(first_step + s) * dt;
                double tau_prev, tau;
                if (options & ORACLE_FAR_FIELD) {
                    tau_prev = radio_oracle_arrival_far(xc, x_prev, t_prev, c);
                    tau = radio_oracle_arrival_far(xc, x_cur, t_cur, c);
                } else {
                    tau_prev = radio_oracle_arrival(xc, x_prev, t_prev, c);
                    tau = radio_oracle_arrival(xc, x_cur, t_cur, c);
                }
                double F[6], Fp[6];
                if (options & ORACLE_HOLD_LINEAR) {
                    /* both ends, each with the centred betadot at its own state */
                    double bd_s[3], bd_p[3];
                    state_betadot(u, n_states, n_p, n_steps, s, p, dt, bd_s);
                    state_betadot(u, n_states, n_p, n_steps, s - 1, p, dt, bd_p);
                    radio_oracle_field_opts(xc, x_cur, beta, g2, bd_s, qp, c, options, F, F + 3);
                    radio_oracle_field_opts(xc, x_prev, beta_prev, g2p, bd_p, qp, c, options, Fp,
                                            Fp + 3);
                } else if (options & ORACLE_HOLD_PREVIOUS) {
                    /* the field of state s-1, with its own backward betadot */
                    double bd_prev[3];
                    if (s >= 2) {
                        double u_pp[3], beta_pp[3], g2pp;
                        load_state(u, n_states, n_p, s - 2, p, u_pp);
                        radio_oracle_kinematics(u_pp, beta_pp, &g2pp);
                        for (int k = 0; k < 3; ++k)
                            bd_prev[k] = (beta_prev[k] - beta_pp[k]) / dt;
                    } else {
                        for (int k = 0; k < 3; ++k)
                            bd_prev[k] = betadot[k];
                    }
                    radio_oracle_field_opts(xc, x_prev, beta_prev, g2p, bd_prev, qp, c, options,
                                            Fp, Fp + 3);
                } else {
                    radio_oracle_field_opts(xc, x_cur, beta, g2, betadot, qp, c, options, F,
                                            F + 3);
                }
                double a = radio_oracle_slot_of(tau_prev, t0, dt_det);
                double b = radio_oracle_slot_of(tau, t0, dt_det);
                double lo = a < b ? a : b;
                double hi = a < b ? b : a;
                if (b < a)
                    ++nonmono;
                if (lo < 0.0 || hi > (double)n_t)
                    ++clipped;
                if (options & ORACLE_HOLD_LINEAR)
                    deposit_interval_linear(Dc, n_t, a, b, Fp, F);
                else if (options & ORACLE_HOLD_PREVIOUS)
                    deposit_interval(Dc, n_t, lo, hi, Fp);
                else
                    deposit_interval(Dc, n_t, lo, hi, F);
            }
        }
    }
    if (counters) {
        counters[0] += clipped;
        counters[1] += nonmono;
    }
    return 0;
}
