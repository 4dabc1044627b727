// Host runtime of libradio: the C interface declared in include/radio.h.
//
// Owns the detector objects (cell positions and the slot accumulator
// resident in device memory), validates every call on the host
// before anything is enqueued, plans the work decomposition and launches the
// kernels on the caller's stream.
#include "radio.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "radio_internal.h"

struct radio_detector {
    int device = 0;
    int n_cus = 1;  // compute units of the device
    int32_t precision = RADIO_FP64;
    int64_t n_c = 0;
    int64_t n_t = 0;
    double t0 = 0.0;
    double dt_det = 1.0;
    double c = 1.0;
    double* d_cells = nullptr;        // internal (tile-ordered) rows
    int64_t* d_user_index = nullptr;  // internal row -> caller's cell index
    double* d_acc = nullptr;
    unsigned long long* d_counters = nullptr;  // [kCounters]: clipped, nonmonotone, ring
                                               // bypasses, large-ring interactions
    char* d_recs = nullptr;                    // workspace (state records), grown on demand
    size_t recs_cap = 0;                       // in bytes
    int32_t* d_perm = nullptr;                 // workspace, grown on demand
    size_t perm_cap = 0;                       // in entries
    uint8_t* d_sel = nullptr;                  // workspace: ring size per tile
    size_t sel_cap = 0;
    int32_t options = 0;                       // RADIO_FAR_FIELD | RADIO_ACCEL_ONLY
    double* d_far = nullptr;                   // FAR_FIELD: [n_c][4] n_cell, R_cell per row
    double2* d_spec = nullptr;                 // spectrum workspace, grown on demand
    size_t spec_cap = 0;                       // in complex values
    int64_t interactions = 0;
    int64_t chunks = 0;
    int64_t slices = 0;  // deposit jobs launched (time slices of single deposits)
    std::vector<double> h_cells;               // caller's order
};

static_assert(RADIO_FP64 == radio::kModeF64 && RADIO_MIXED == radio::kModeMix &&
                  RADIO_MIXED_TWOSUM == radio::kModeMixTwoSum,
              "precision codes double as kernel modes");

namespace {

// launch tunables (radio_set_tuning)
std::mutex g_tuning_mu;
radio_tuning g_tuning = {0, 4, 1 << 22, 0, 0};

radio_tuning current_tuning()
{
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    return g_tuning;
}

bool finite3(const double v[3])
{
    return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

double norm3(const double v[3])
{
    return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
}

// cell positions of the generated geometries (radio.h documents the formulas)
int build_cells(const radio_detector_desc& d, std::vector<double>& out)
{
    if (d.geometry == RADIO_GEOM_EXPLICIT) {
        if (d.n_cells < 1 || !d.cells)
            return RADIO_EINVAL;
        out.assign(d.cells, d.cells + 3 * d.n_cells);
        for (double v : out)
            if (!std::isfinite(v))
                return RADIO_EINVAL;
        return RADIO_OK;
    }
    if (d.n1 < 1 || d.n2 < 1 || d.n1 > (int64_t)1 << 20 || d.n2 > (int64_t)1 << 20)
        return RADIO_EINVAL;
    if (!std::isfinite(d.half1) || !std::isfinite(d.half2) || d.half1 < 0.0 || d.half2 < 0.0)
        return RADIO_EINVAL;
    const int64_t n1 = d.n1, n2 = d.n2;
    const int64_t n3 = d.n3 > 0 ? d.n3 : 1;  // spherical shells
    if (d.geometry != RADIO_GEOM_SPHERE && n3 != 1)
        return RADIO_EINVAL;
    if (n3 > 4096 || n1 * n2 * n3 > (int64_t)1 << 32)
        return RADIO_EINVAL;
    out.resize((size_t)(3 * n1 * n2 * n3));
    if (d.geometry == RADIO_GEOM_PLANE) {
        if (!finite3(d.origin) || !finite3(d.e1) || !finite3(d.e2))
            return RADIO_EINVAL;
        const double l1 = norm3(d.e1), l2 = norm3(d.e2);
        if (!(l1 > 0.0) || !(l2 > 0.0))
            return RADIO_EINVAL;
        const double e1[3] = {d.e1[0] / l1, d.e1[1] / l1, d.e1[2] / l1};
        const double e2[3] = {d.e2[0] / l2, d.e2[1] / l2, d.e2[2] / l2};
        for (int64_t i2 = 0; i2 < n2; ++i2) {
            const double a2 = -d.half2 + ((double)i2 + 0.5) * (2.0 * d.half2 / (double)n2);
            for (int64_t i1 = 0; i1 < n1; ++i1) {
                const double a1 = -d.half1 + ((double)i1 + 0.5) * (2.0 * d.half1 / (double)n1);
                double* p = &out[(size_t)(3 * (i2 * n1 + i1))];
                for (int k = 0; k < 3; ++k)
                    p[k] = d.origin[k] + a1 * e1[k] + a2 * e2[k];
            }
        }
        return RADIO_OK;
    }
    if (d.geometry == RADIO_GEOM_SPHERE) {
        if (!finite3(d.axis) || !finite3(d.e1) || !(d.radius > 0.0) || !std::isfinite(d.radius) ||
            !std::isfinite(d.radius_step) || !(d.radius + (double)(n3 - 1) * d.radius_step > 0.0))
            return RADIO_EINVAL;
        const double la = norm3(d.axis);
        if (!(la > 0.0))
            return RADIO_EINVAL;
        const double ax[3] = {d.axis[0] / la, d.axis[1] / la, d.axis[2] / la};
        const double pr = d.e1[0] * ax[0] + d.e1[1] * ax[1] + d.e1[2] * ax[2];
        double e1[3] = {d.e1[0] - pr * ax[0], d.e1[1] - pr * ax[1], d.e1[2] - pr * ax[2]};
        const double l1 = norm3(e1);
        if (!(l1 > 1e-12 * norm3(d.e1)))
            return RADIO_EINVAL;
        for (double& v : e1)
            v /= l1;
        const double e2[3] = {ax[1] * e1[2] - ax[2] * e1[1], ax[2] * e1[0] - ax[0] * e1[2],
                              ax[0] * e1[1] - ax[1] * e1[0]};
        for (int64_t i3 = 0; i3 < n3; ++i3) {
            const double radius = d.radius + (double)i3 * d.radius_step;
            for (int64_t i2 = 0; i2 < n2; ++i2) {
                const double lat = -d.half2 + ((double)i2 + 0.5) * (2.0 * d.half2 / (double)n2);
                for (int64_t i1 = 0; i1 < n1; ++i1) {
                    const double lon =
                        -d.half1 + ((double)i1 + 0.5) * (2.0 * d.half1 / (double)n1);
                    double* p = &out[(size_t)(3 * ((i3 * n2 + i2) * n1 + i1))];
                    for (int k = 0; k < 3; ++k)
                        p[k] = radius * (std::cos(lat) * (std::cos(lon) * ax[k] +
                                                          std::sin(lon) * e1[k]) +
                                         std::sin(lat) * e2[k]);
                }
            }
        }
        return RADIO_OK;
    }
    return RADIO_EINVAL;
}

// Order the cells so that tiles of consecutive rows are compact in direction
// (as seen from the origin, where the radiating particles are expected): a
// Morton code of each cell's direction projected on the plane normal to the
// mean direction.  Cells with similar directions see similar arrival-time
// offsets between particles, which is what the deposit's slot rings rely on.
std::vector<int64_t> order_cells(const std::vector<double>& cells, int64_t per_group)
{
    const int64_t n = (int64_t)(cells.size() / 3);
    std::vector<double> dir(3 * n, 0.0);
    double m[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        const double* c = &cells[3 * i];
        const double l = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        if (l > 0.0)
            for (int k = 0; k < 3; ++k) {
                dir[3 * i + k] = c[k] / l;
                m[k] += c[k] / l;
            }
    }
    double lm = norm3(m);
    if (!(lm > 1e-12 * (double)n)) {
        m[0] = 0.0;
        m[1] = 0.0;
        m[2] = 1.0;
        lm = 1.0;
    }
    for (double& v : m)
        v /= lm;
    // e1 orthogonal to m, e2 = m x e1
    double t[3] = {1.0, 0.0, 0.0};
    if (std::fabs(m[0]) > 0.9) {
        t[0] = 0.0;
        t[1] = 1.0;
    }
    const double pr = t[0] * m[0] + t[1] * m[1] + t[2] * m[2];
    double e1[3] = {t[0] - pr * m[0], t[1] - pr * m[1], t[2] - pr * m[2]};
    const double l1 = norm3(e1);
    for (double& v : e1)
        v /= l1;
    const double e2[3] = {m[1] * e1[2] - m[2] * e1[1], m[2] * e1[0] - m[0] * e1[2],
                          m[0] * e1[1] - m[1] * e1[0]};
    std::vector<double> a(n), b(n);
    double amin = 1e300, amax = -1e300, bmin = 1e300, bmax = -1e300;
    for (int64_t i = 0; i < n; ++i) {
        const double* d = &dir[3 * i];
        a[i] = d[0] * e1[0] + d[1] * e1[1] + d[2] * e1[2];
        b[i] = d[0] * e2[0] + d[1] * e2[1] + d[2] * e2[2];
        amin = std::min(amin, a[i]);
        amax = std::max(amax, a[i]);
        bmin = std::min(bmin, b[i]);
        bmax = std::max(bmax, b[i]);
    }
    const double sa = amax > amin ? 65535.0 / (amax - amin) : 0.0;
    const double sb = bmax > bmin ? 65535.0 / (bmax - bmin) : 0.0;
    std::vector<uint64_t> code(n);
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t qa = (uint32_t)std::lround((a[i] - amin) * sa);
        const uint32_t qb = (uint32_t)std::lround((b[i] - bmin) * sb);
        uint64_t c = 0;
        for (int bit = 0; bit < 16; ++bit)
            c |= ((uint64_t)((qa >> bit) & 1u) << (2 * bit)) |
                 ((uint64_t)((qb >> bit) & 1u) << (2 * bit + 1));
        code[i] = c;
    }
    std::vector<int64_t> idx(n);
    std::iota(idx.begin(), idx.end(), (int64_t)0);
    // cells of one group (a spherical shell) stay together: their arrival times differ
    // from another shell's by the radial distance
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
        const int64_t gx = x / per_group, gy = y / per_group;
        return gx != gy ? gx < gy : code[x] < code[y];
    });
    return idx;
}

// Make det's device current for the duration of a call, restoring the caller's.
class DeviceGuard {
  public:
    explicit DeviceGuard(int dev) : ok_(true)
    {
        if (hipGetDevice(&prev_) != hipSuccess) {
            ok_ = false;
            return;
        }
        if (prev_ != dev && hipSetDevice(dev) != hipSuccess)
            ok_ = false;
        target_ = dev;
    }
    ~DeviceGuard()
    {
        if (ok_ && prev_ != target_)
            (void)hipSetDevice(prev_);
    }
    bool ok() const { return ok_; }

  private:
    int prev_ = 0;
    int target_ = 0;
    bool ok_;
};

int validate_chunk(const radio_chunk* k)
{
    if (!k)
        return RADIO_EINVAL;
    if (k->n_particles < 0 || k->n_steps < 0)
        return RADIO_EINVAL;
    if (k->first_step < 0 || k->first_step > (INT64_C(1) << 53) - 1 - k->n_steps)
        return RADIO_EINVAL;
    if (!std::isfinite(k->t_first) || !std::isfinite(k->dt) || !(k->dt > 0.0))
        return RADIO_EINVAL;
    if (k->n_particles == 0 || k->n_steps == 0)
        return RADIO_OK;
    if (!k->x || !k->u)
        return RADIO_EINVAL;
    // keep every flattened index inside int64
    const double states = (double)k->n_steps + 1.0;
    if (3.0 * states * (double)k->n_particles > 9.0e18)
        return RADIO_EINVAL;
    return RADIO_OK;
}

// The far-field geometry of every cell (Eq. 3): its direction n = x * (1/R) and
// distance R = sqrt(|x|^2) from the origin, as [n0, n1, n2, R] per row, one IEEE
// operation at a time (these enter the arrival time).  False if a cell sits
// at the origin.
bool far_geometry(const std::vector<double>& cells, std::vector<double>& far)
{
#pragma clang fp contract(off)
    const size_t n = cells.size() / 3;
    far.resize(4 * n);
    for (size_t r = 0; r < n; ++r) {
        const double* x = &cells[3 * r];
        const double R = std::sqrt((x[0] * x[0] + x[1] * x[1]) + x[2] * x[2]);
        if (!(R > 0.0) || !std::isfinite(R))
            return false;
        const double ri = 1.0 / R;
        far[4 * r] = x[0] * ri;
        far[4 * r + 1] = x[1] * ri;
        far[4 * r + 2] = x[2] * ri;
        far[4 * r + 3] = R;
    }
    return true;
}

radio::DepositJob make_job(const radio_detector* det, const radio_chunk* k)
{
    radio::DepositJob J{};
    J.cells = det->d_cells;
    J.acc = det->d_acc;
    J.counters = det->d_counters;
    J.x = k->x;
    J.u = k->u;
    J.q = k->q;
    J.n_c = det->n_c;
    J.n_t = det->n_t;
    J.n_p = k->n_particles;
    J.n_s = k->n_steps;
    J.t_first = k->t_first;
    J.s0 = k->first_step;
    J.xs_stride = (k->n_steps + 1) * k->n_particles;
    J.s_before = 0;
    J.s_after = 0;
    J.far = det->d_far;
    J.vscale = (det->options & RADIO_ACCEL_ONLY) ? 0.0 : 1.0;
    J.hold = (det->options & RADIO_HOLD_LINEAR) ? 2 : ((det->options & RADIO_HOLD_PREVIOUS) ? 1 : 0);
    J.potentials = (det->options & RADIO_POTENTIALS) ? 1 : 0;
    J.dt = k->dt;
    J.t0 = det->t0;
    J.inv_dt_det = 1.0 / det->dt_det;  // correctly rounded (host IEEE division)
    J.dt_det = det->dt_det;
    J.slot_div = radio::slot_quotient_corrects(det->dt_det) ? 0 : 1;
    J.inv_c = 1.0 / det->c;
    J.c = det->c;
    // the tuned workgroup shape, for detectors with the default options (the
    // other shapes are compiled for those only)
    const int shape = current_tuning().shape;
    radio::set_shape(J, (det->options == 0 && shape > 0 && shape < radio::kShapes) ? shape : 0);
    const int per_cu =
        radio::persistent_blocks_per_cu(radio::kernel_variant(det->precision, J), false);
    radio::plan_job(J, current_tuning().target_blocks, (int64_t)det->n_cus * per_cu);
    radio::set_groups(J, radio::max_order_groups(J, radio::rec_bytes(det->precision),
                                                 current_tuning().order_budget_mib));
    return J;
}

// The job of the time slice [r_a, r_b) of the runs of the whole-chunk job W:
// its states, with the neighbours the kinematics reads, and its own work
// decomposition, with at most max_groups particle orders.
radio::DepositJob slice_job(const radio_detector* det, const radio::DepositJob& W, int64_t r_a,
                            int64_t r_b, int64_t max_groups)
{
    radio::DepositJob J = W;
    const int64_t a = r_a * W.run_l;
    const int64_t b = std::min(r_b * W.run_l, W.n_s);
    J.x = W.x + a * W.n_p;
    J.u = W.u + a * W.n_p;
    J.n_s = b - a;
    J.s0 = W.s0 + a;
    J.s_before = W.s_before + a;
    J.s_after = W.s_after + (W.n_s - b);
    const int per_cu =
        radio::persistent_blocks_per_cu(radio::kernel_variant(det->precision, J), false);
    radio::plan_job(J, current_tuning().target_blocks, (int64_t)det->n_cus * per_cu);
    radio::set_groups(J, max_groups);
    return J;
}

// Grow a device workspace to hold at least `need` elements, in stream order on
// s: the old buffer is released with hipFreeAsync once s has passed the work
// already enqueued on it (the previous user of a detector's workspace is
// ordered before s by the caller; a batch arena's previous batch has been
// waited for), and the new one comes from the device's stream-ordered pool.
// Nothing waits on the host and no other stream is stalled.
template <typename T>
int grow(T** p, size_t* cap, size_t need, hipStream_t s)
{
    if (need <= *cap)
        return RADIO_OK;
    if (*p) {
        if (hipFreeAsync(*p, s) != hipSuccess)
            return RADIO_EDEVICE;
        *p = nullptr;
        *cap = 0;
    }
    if (hipMallocAsync((void**)p, need * sizeof(T), s) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return RADIO_ENOMEM;
    }
    *cap = need;
    return RADIO_OK;
}

// Release a workspace of grow() (the device is idle: destroy synchronises first).
template <typename T>
void release(T** p, size_t* cap)
{
    if (*p)
        (void)hipFreeAsync(*p, nullptr);
    *p = nullptr;
    *cap = 0;
}

// The time slices of one deposit: a chunk whose particle orders of at most
// kRunsPerGroup runs would not fit the order budget is deposited in time slices
// that each do.  The slices share the state-time origin and read their
// neighbour states, so that the sum of their deposits is the chunk's, up to
// summation order.  The first slice is the largest.
struct SlicePlan {
    radio::DepositJob W;  // the whole chunk
    int64_t max_groups = 0;
    int64_t n_slices = 1;
    int64_t runs_each = 0;
};

SlicePlan plan_slices(const radio_detector* det, const radio_chunk* k)
{
    SlicePlan P;
    P.W = make_job(det, k);
    P.max_groups = radio::max_order_groups(P.W, radio::rec_bytes(det->precision),
                                           current_tuning().order_budget_mib);
    const bool slice = P.W.n_p >= radio::min_group_particles(P.W) &&
                       P.W.runs_per_group > radio::kRunsPerGroup;
    const int64_t slice_runs = slice ? P.max_groups * radio::kRunsPerGroup : P.W.n_runs;
    P.n_slices = (P.W.n_runs + slice_runs - 1) / slice_runs;
    P.runs_each = (P.W.n_runs + P.n_slices - 1) / P.n_slices;
    return P;
}

radio::DepositJob plan_slice(const radio_detector* det, const SlicePlan& P, int64_t r_a)
{
    if (P.n_slices == 1)
        return P.W;
    return slice_job(det, P.W, r_a, std::min(r_a + P.runs_each, P.W.n_runs), P.max_groups);
}

// Grow the detector's workspaces to hold slice job J (stream-ordered on s).
int reserve(radio_detector* det, const radio::DepositJob& J, hipStream_t s)
{
    int rc = grow(&det->d_recs, &det->recs_cap,
                  (size_t)(J.n_p * (J.n_s + 1)) * radio::rec_bytes(det->precision), s);
    if (rc == RADIO_OK)
        rc = grow(&det->d_perm, &det->perm_cap, (size_t)(J.n_groups * J.n_tiles * J.n_p), s);
    if (rc == RADIO_OK)
        rc = grow(&det->d_sel, &det->sel_cap, (size_t)J.n_tiles, s);
    return rc;
}

// Enqueue a deposit in its time slices.  Only the first (largest) slice can
// grow the workspaces, so a later one cannot fail for memory after earlier
// ones were enqueued.
int enqueue_deposit(radio_detector* det, const radio_chunk* k, hipStream_t s)
{
    if (k->n_particles == 0 || k->n_steps == 0)
        return RADIO_OK;
    if (k->n_particles > INT32_MAX || k->n_steps > INT32_MAX - 1)
        return RADIO_EINVAL;
    const SlicePlan P = plan_slices(det, k);
    for (int64_t r_a = 0; r_a < P.W.n_runs; r_a += P.runs_each) {
        radio::DepositJob J = plan_slice(det, P, r_a);
        const int rc = reserve(det, J, s);
        if (rc != RADIO_OK)
            return rc;
        J.recs = det->d_recs;
        J.perm = det->d_perm;
        J.ring_sel = det->d_sel;
        if (radio::launch_kinematics(J, det->precision, s) != hipSuccess ||
            radio::launch_order(J, s) != hipSuccess ||
            radio::launch_ring_choice(J, det->precision, s) != hipSuccess ||
            radio::launch_deposit(J, det->precision, current_tuning().max_grid, s) != hipSuccess)
            return RADIO_EDEVICE;
        det->slices += 1;
    }
    det->interactions += k->n_particles * k->n_steps * det->n_c;
    return RADIO_OK;
}

// ---------------------------------------------------------------------------
// The deposit that allocates nothing: its workspaces (state records, particle
// orders, ring choices) live in one fixed device array per GPU, `scratch`.
// Every call on a GPU shares that GPU's copy; calls on one stream follow each
// other, calls that overlap on one GPU (different streams) race.  Nothing in it
// needs clearing: each launch's kinematics, order and ring-choice kernels write
// every word the deposit kernel of the same launch reads.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// The device address of this GPU's scratch, looked up once per device with that
// device current (the array's name is no device address in host code).
int scratch_of(int dev, char** out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return RADIO_ESTATE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return RADIO_EDEVICE;
        }
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return RADIO_OK;
}

constexpr size_t align256(size_t n)
{
    return (n + 255) / 256 * 256;
}

// Bytes of the scratch a time slice of `runs` runs of job W takes: its records
// (with their one-state overlap), one order per kRunsPerGroup runs, ring choices.
size_t slice_scratch_bytes(const radio::DepositJob& W, int precision, int64_t runs)
{
    const int64_t states = std::min(runs * W.run_l, W.n_s) + 1;
    const int64_t groups = W.n_p < radio::min_group_particles(W)
                               ? 1
                               : (runs + radio::kRunsPerGroup - 1) / radio::kRunsPerGroup;
    return align256((size_t)(W.n_p * states) * radio::rec_bytes(precision)) +
           align256((size_t)(groups * W.n_tiles * W.n_p) * sizeof(int32_t)) +
           align256((size_t)W.n_tiles);
}

int enqueue_deposit_noalloc(radio_detector* det, const radio_chunk* k, hipStream_t s)
{
    if (k->n_particles == 0 || k->n_steps == 0)
        return RADIO_OK;
    if (k->n_particles > INT32_MAX || k->n_steps > INT32_MAX - 1)
        return RADIO_EINVAL;
    char* base = nullptr;
    int rc = scratch_of(det->device, &base);
    if (rc != RADIO_OK)
        return rc;
    const radio::DepositJob W = make_job(det, k);
    if (slice_scratch_bytes(W, det->precision, 1) > kScratchBytes)
        return RADIO_ETOOBIG;
    // the longest time slices that fit the scratch
    int64_t lo = 1, hi = W.n_runs;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (slice_scratch_bytes(W, det->precision, mid) <= kScratchBytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int64_t n_slices = (W.n_runs + lo - 1) / lo;
    const int64_t runs_each = (W.n_runs + n_slices - 1) / n_slices;
    const int64_t groups_each = (runs_each + radio::kRunsPerGroup - 1) / radio::kRunsPerGroup;
    for (int64_t r_a = 0; r_a < W.n_runs; r_a += runs_each) {
        radio::DepositJob J =
            slice_job(det, W, r_a, std::min(r_a + runs_each, W.n_runs), groups_each);
        const size_t rec_b = align256((size_t)(J.n_p * (J.n_s + 1)) * radio::rec_bytes(det->precision));
        const size_t perm_b = align256((size_t)(J.n_groups * J.n_tiles * J.n_p) * sizeof(int32_t));
        if (rec_b + perm_b + align256((size_t)J.n_tiles) > kScratchBytes)
            return RADIO_ETOOBIG;  // not reached: the slices were sized to fit
        J.recs = base;
        J.perm = reinterpret_cast<int32_t*>(base + rec_b);
        J.ring_sel = reinterpret_cast<uint8_t*>(base + rec_b + perm_b);
        if (radio::launch_kinematics(J, det->precision, s) != hipSuccess ||
            radio::launch_order(J, s) != hipSuccess ||
            radio::launch_ring_choice(J, det->precision, s) != hipSuccess ||
            radio::launch_deposit(J, det->precision, current_tuning().max_grid, s) != hipSuccess)
            return RADIO_EDEVICE;
        det->slices += 1;
    }
    det->interactions += k->n_particles * k->n_steps * det->n_c;
    return RADIO_OK;
}

// Workspaces of batched deposits, per device: every pair of a batch needs its
// own state records and particle orders until the persistent launch has run, so
// they come from one arena; before the arena is reused the previous batch's
// event is waited for.
struct BatchArena {
    radio::DepositJob* d_jobs = nullptr;
    size_t jobs_cap = 0;
    radio::WorkItem* d_items = nullptr;
    size_t items_cap = 0;
    unsigned long long* d_next = nullptr;  // two counters (ring sizes) per kernel variant
    char* d_recs = nullptr;  // state records of every pair, in bytes
    size_t recs_cap = 0;
    int32_t* d_perm = nullptr;
    size_t perm_cap = 0;
    uint8_t* d_sel = nullptr;
    size_t sel_cap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
    std::vector<radio::DepositJob> h_jobs;
    std::vector<radio::WorkItem> h_items;
    int n_cus = 0;
};

// Two arenas per device, used in turn: a batch can be prepared and enqueued
// while the previous one still runs, and only the batch before that must have
// finished.
constexpr int kArenas = 2;
constexpr int kVariants = radio::kKernelVariants;
std::mutex g_arena_mu;
std::map<int, BatchArena*> g_arenas[kArenas];
std::map<int, int> g_arena_next;

int enqueue_batch(radio_detector* const* dets, const radio_chunk* chunks, int n, hipStream_t s,
                  int dev)
{
    std::lock_guard<std::mutex> lk(g_arena_mu);
    const int which = g_arena_next[dev];
    g_arena_next[dev] = (which + 1) % kArenas;
    BatchArena*& A = g_arenas[which][dev];
    if (!A) {
        A = new (std::nothrow) BatchArena();
        if (!A)
            return RADIO_ENOMEM;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess ||
            hipEventCreateWithFlags(&A->done, hipEventDisableTiming) != hipSuccess ||
            hipMalloc((void**)&A->d_next, 2 * kVariants * sizeof(unsigned long long)) != hipSuccess) {
            (void)hipGetLastError();
            return RADIO_EDEVICE;
        }
        A->n_cus = prop.multiProcessorCount;
    }
    if (A->pending) {
        if (hipEventSynchronize(A->done) != hipSuccess)
            return RADIO_EDEVICE;
        A->pending = false;
    }
    // Plan every nonempty pair.  A pair whose particle orders would not fit the
    // order budget is deposited after the persistent launch, in the time slices
    // of a single deposit on its detector's own workspaces; those are grown
    // here, before anything is enqueued, so that a memory error leaves every
    // detector as it was.
    const radio_tuning tun = current_tuning();
    std::vector<int> idx, sliced;
    size_t recs_need = 0, perm_need = 0, sel_need = 0;
    A->h_jobs.clear();
    for (int i = 0; i < n; ++i) {
        const radio_chunk* k = &chunks[i];
        if (k->n_particles == 0 || k->n_steps == 0)
            continue;
        const SlicePlan P = plan_slices(dets[i], k);
        if (P.n_slices > 1) {
            const int rc = reserve(dets[i], plan_slice(dets[i], P, 0), s);
            if (rc != RADIO_OK)
                return rc;
            sliced.push_back(i);
            continue;
        }
        const radio::DepositJob& J = P.W;
        recs_need += (size_t)(J.n_p * (J.n_s + 1)) * radio::rec_bytes(dets[i]->precision);
        perm_need += (size_t)(J.n_groups * J.n_tiles * J.n_p);
        sel_need += (size_t)J.n_tiles;
        A->h_jobs.push_back(J);
        idx.push_back(i);
    }
    if (idx.empty()) {
        for (int i : sliced) {
            const int rc = enqueue_deposit(dets[i], &chunks[i], s);
            if (rc != RADIO_OK)
                return rc;
        }
        for (int i = 0; i < n; ++i)
            dets[i]->chunks += 1;
        return RADIO_OK;
    }
    int rc = grow(&A->d_recs, &A->recs_cap, recs_need, s);
    if (rc == RADIO_OK)
        rc = grow(&A->d_perm, &A->perm_cap, perm_need, s);
    if (rc == RADIO_OK)
        rc = grow(&A->d_sel, &A->sel_cap, sel_need, s);
    if (rc == RADIO_OK)
        rc = grow(&A->d_jobs, &A->jobs_cap, A->h_jobs.size(), s);
    if (rc != RADIO_OK)
        return rc;
    // work items: a per-pair split chosen so that items carry similar work, longest first
    double total = 0.0;
    for (const auto& J : A->h_jobs)
        total += (double)J.n_c * (double)J.n_p * (double)J.n_s;
    int bpc[kVariants][2];  // resident workgroups per CU: [variant][large ring]
    for (int v = 0; v < kVariants; ++v)
        for (int r = 0; r < 2; ++r)
            bpc[v][r] = radio::persistent_blocks_per_cu(v, r == 1);
    const double resident = (double)A->n_cus * (double)bpc[0][0];
    const double item_work = std::max(total / (resident * (double)tun.items_per_workgroup), 1.0);
    struct Item {
        radio::WorkItem w;
        double cost;
        int mode;
    };
    std::vector<Item> items;
    size_t ro = 0, po = 0, so = 0;
    for (size_t j = 0; j < A->h_jobs.size(); ++j) {
        radio::DepositJob& J = A->h_jobs[j];
        const int prec = dets[idx[j]]->precision;
        J.recs = A->d_recs + ro;
        J.perm = A->d_perm + po;
        J.ring_sel = A->d_sel + so;
        ro += (size_t)(J.n_p * (J.n_s + 1)) * radio::rec_bytes(prec);
        po += (size_t)(J.n_groups * J.n_tiles * J.n_p);
        so += (size_t)J.n_tiles;
        const double run_work = (double)J.tile_cells * (double)J.n_p * (double)J.run_l;
        // items of similar work, and short (see kMinItemBatches)
        const int64_t n_batches = (J.n_p + J.groups - 1) / J.groups;
        const int64_t rps_short = (radio::kMinItemBatches + n_batches - 1) / n_batches;
        int64_t rps = std::min<int64_t>((int64_t)std::ceil(item_work / run_work), rps_short);
        rps = std::max<int64_t>(1, std::min<int64_t>(rps, J.n_runs));
        J.runs_per_split = rps;
        J.n_splits = (J.n_runs + rps - 1) / rps;
        radio::set_parts(J, 1);  // batch items cover all of a tile's particles
        const int mode = radio::kernel_variant(prec, J);  // kernel variant
        for (int64_t sp = 0; sp < J.n_splits; ++sp) {
            const int64_t runs = std::min<int64_t>(rps, J.n_runs - sp * rps);
            for (int64_t t = 0; t < J.n_tiles; ++t)
                items.push_back({{(int32_t)j, (int32_t)t, (int32_t)sp, 0},
                                 (double)runs * run_work, mode});
        }
        if (radio::launch_kinematics(J, prec, s) != hipSuccess ||
            radio::launch_order(J, s) != hipSuccess ||
            radio::launch_ring_choice(J, prec, s) != hipSuccess)
            return RADIO_EDEVICE;
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) {
        return a.mode != b.mode ? a.mode < b.mode : a.cost > b.cost;
    });
    A->h_items.resize(items.size());
    for (size_t i = 0; i < items.size(); ++i)
        A->h_items[i] = items[i].w;
    rc = grow(&A->d_items, &A->items_cap, A->h_items.size(), s);
    if (rc != RADIO_OK)
        return rc;
    if (hipMemcpyAsync(A->d_jobs, A->h_jobs.data(), A->h_jobs.size() * sizeof(radio::DepositJob),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(A->d_items, A->h_items.data(), A->h_items.size() * sizeof(radio::WorkItem),
                       hipMemcpyHostToDevice, s) != hipSuccess)
        return RADIO_EDEVICE;
    size_t b = 0;
    while (b < items.size()) {
        const int mode = items[b].mode;
        size_t e = b;
        while (e < items.size() && items[e].mode == mode)
            ++e;
        if (radio::launch_deposit_batch(A->d_jobs, A->d_items + b, (int64_t)(e - b),
                                        A->d_next + 2 * mode, mode, A->n_cus * bpc[mode][0],
                                        A->n_cus * bpc[mode][1], s) != hipSuccess)
            return RADIO_EDEVICE;
        b = e;
    }
    if (hipEventRecord(A->done, s) != hipSuccess)
        return RADIO_EDEVICE;
    A->pending = true;
    for (size_t j = 0; j < idx.size(); ++j) {
        const radio_chunk* k = &chunks[idx[j]];
        dets[idx[j]]->interactions += k->n_particles * k->n_steps * dets[idx[j]]->n_c;
        dets[idx[j]]->slices += 1;
    }
    for (int i : sliced) {
        rc = enqueue_deposit(dets[i], &chunks[i], s);
        if (rc != RADIO_OK)
            return rc;
    }
    for (int i = 0; i < n; ++i)
        dets[i]->chunks += 1;
    return RADIO_OK;
}

}  // namespace

namespace radio {

bool slot_quotient_corrects(double b)
{
    if (!(b >= 0x1p-900 && b <= 0x1p900))
        return false;
    const double y = 1.0 / b;                // RN(1/b)
    const double e = std::fma(b, y, -1.0);   // b y - 1, exact
    int ex = 0;
    const double B = std::ldexp(std::frexp(b, &ex), 53);  // integer in [2^52, 2^53)
    return std::fabs(e) * B < 1.0 - 0x1p-45;
}

}  // namespace radio

extern "C" {

const char* radio_status_string(int status)
{
    switch (status) {
    case RADIO_OK:
        return "ok";
    case RADIO_EINVAL:
        return "invalid argument";
    case RADIO_ENOMEM:
        return "out of memory";
    case RADIO_EDEVICE:
        return "device error";
    case RADIO_ESTATE:
        return "invalid state";
    case RADIO_ETOOBIG:
        return "chunk too large for the fixed scratch of the non-allocating deposit";
    default:
        return "unknown status";
    }
}

int radio_detector_create(const radio_detector_desc* desc, void* stream, radio_detector** out)
{
    if (!desc || !out)
        return RADIO_EINVAL;
    if (desc->precision != RADIO_FP64 && desc->precision != RADIO_MIXED &&
        desc->precision != RADIO_MIXED_TWOSUM)
        return RADIO_EINVAL;
    if (!std::isfinite(desc->t0) || !std::isfinite(desc->dt_det) || !(desc->dt_det > 0.0) ||
        !std::isfinite(1.0 / desc->dt_det))
        return RADIO_EINVAL;
    if (desc->n_t < 1 || desc->n_t > (int64_t)1 << 30)
        return RADIO_EINVAL;
    if (!std::isfinite(desc->c) || !(desc->c > 0.0))
        return RADIO_EINVAL;
    if ((desc->options & ~(RADIO_FAR_FIELD | RADIO_ACCEL_ONLY | RADIO_HOLD_PREVIOUS |
                           RADIO_HOLD_LINEAR | RADIO_POTENTIALS)) != 0 ||
        ((desc->options & RADIO_HOLD_PREVIOUS) && (desc->options & RADIO_HOLD_LINEAR)) ||
        ((desc->options & RADIO_POTENTIALS) && (desc->options & RADIO_ACCEL_ONLY)))
        return RADIO_EINVAL;
    std::vector<double> cells;
    int rc = build_cells(*desc, cells);
    if (rc != RADIO_OK)
        return rc;
    const int64_t n_c = (int64_t)(cells.size() / 3);
    if ((double)n_c * (double)desc->n_t * 6.0 > 4.0e18)
        return RADIO_EINVAL;

    radio_detector* det = new (std::nothrow) radio_detector();
    if (!det)
        return RADIO_ENOMEM;
    if (hipGetDevice(&det->device) != hipSuccess ||
        hipDeviceGetAttribute(&det->n_cus, hipDeviceAttributeMultiprocessorCount, det->device) !=
            hipSuccess) {
        (void)hipGetLastError();
        delete det;
        return RADIO_EDEVICE;
    }
    det->precision = desc->precision;
    det->options = desc->options;
    det->n_c = n_c;
    det->n_t = desc->n_t;
    det->t0 = desc->t0;
    det->dt_det = desc->dt_det;
    det->c = desc->c;
    det->h_cells.swap(cells);
    hipStream_t s = (hipStream_t)stream;
    const int64_t per_shell =
        (desc->geometry == RADIO_GEOM_SPHERE && desc->n3 > 1) ? n_c / desc->n3 : n_c;
    const std::vector<int64_t> user = order_cells(det->h_cells, per_shell);
    std::vector<double> internal((size_t)(3 * n_c));
    for (int64_t r = 0; r < n_c; ++r)
        for (int k = 0; k < 3; ++k)
            internal[(size_t)(3 * r + k)] = det->h_cells[(size_t)(3 * user[(size_t)r] + k)];
    const size_t acc_bytes = (size_t)n_c * (size_t)det->n_t * 6 * sizeof(double);
    if (hipMalloc((void**)&det->d_acc, acc_bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete det;
        return RADIO_ENOMEM;
    }
    if (hipMalloc((void**)&det->d_cells, (size_t)n_c * 3 * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&det->d_user_index, (size_t)n_c * sizeof(int64_t)) != hipSuccess ||
        hipMalloc((void**)&det->d_counters, radio::kCounters * sizeof(unsigned long long)) != hipSuccess) {
        (void)hipGetLastError();
        radio_detector_destroy(det);
        return RADIO_ENOMEM;
    }
    std::vector<double> far;
    if (det->options & RADIO_FAR_FIELD) {
        if (!far_geometry(internal, far)) {  // a cell at the origin has no direction
            radio_detector_destroy(det);
            return RADIO_EINVAL;
        }
        if (hipMalloc((void**)&det->d_far, far.size() * sizeof(double)) != hipSuccess ||
            hipMemcpyAsync(det->d_far, far.data(), far.size() * sizeof(double),
                           hipMemcpyHostToDevice, s) != hipSuccess) {
            (void)hipGetLastError();
            radio_detector_destroy(det);
            return RADIO_ENOMEM;
        }
    }
    if (hipMemcpyAsync(det->d_cells, internal.data(), (size_t)n_c * 3 * sizeof(double),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(det->d_user_index, user.data(), (size_t)n_c * sizeof(int64_t),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        radio::launch_zero(det->d_acc, n_c * det->n_t * 6, s) != hipSuccess ||
        radio::launch_zero_u64(det->d_counters, radio::kCounters, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {  // the host vectors are pageable: finish
        radio_detector_destroy(det);
        return RADIO_EDEVICE;
    }
    *out = det;
    return RADIO_OK;
}

int radio_detector_destroy(radio_detector* det)
{
    if (!det)
        return RADIO_OK;
    int rc = RADIO_OK;
    {
        DeviceGuard g(det->device);
        if (!g.ok())
            rc = RADIO_EDEVICE;
        if (hipDeviceSynchronize() != hipSuccess)
            rc = RADIO_EDEVICE;
        if (det->d_acc)
            (void)hipFree(det->d_acc);
        if (det->d_cells)
            (void)hipFree(det->d_cells);
        if (det->d_user_index)
            (void)hipFree(det->d_user_index);
        if (det->d_counters)
            (void)hipFree(det->d_counters);
        release(&det->d_recs, &det->recs_cap);
        release(&det->d_perm, &det->perm_cap);
        release(&det->d_sel, &det->sel_cap);
        release(&det->d_spec, &det->spec_cap);
        if (det->d_far)
            (void)hipFree(det->d_far);
        if (hipStreamSynchronize(nullptr) != hipSuccess)
            rc = RADIO_EDEVICE;
    }
    delete det;
    return rc;
}

int radio_detector_reset(radio_detector* det, void* stream)
{
    if (!det)
        return RADIO_EINVAL;
    DeviceGuard g(det->device);
    if (!g.ok())
        return RADIO_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    if (radio::launch_zero(det->d_acc, det->n_c * det->n_t * 6, s) != hipSuccess ||
        radio::launch_zero_u64(det->d_counters, radio::kCounters, s) != hipSuccess)
        return RADIO_EDEVICE;
    det->interactions = 0;
    det->chunks = 0;
    det->slices = 0;
    return RADIO_OK;
}

int radio_deposit_trajectory_chunk(radio_detector* det, const radio_chunk* chunk, void* stream)
{
    if (!det)
        return RADIO_EINVAL;
    int rc = validate_chunk(chunk);
    if (rc != RADIO_OK)
        return rc;
    DeviceGuard g(det->device);
    if (!g.ok())
        return RADIO_EDEVICE;
    rc = enqueue_deposit(det, chunk, (hipStream_t)stream);
    if (rc == RADIO_OK)
        det->chunks += 1;
    return rc;
}

int radio_deposit_trajectory_chunk_noalloc(radio_detector* det, const radio_chunk* chunk,
                                           void* stream)
{
    if (!det)
        return RADIO_EINVAL;
    int rc = validate_chunk(chunk);
    if (rc != RADIO_OK)
        return rc;
    DeviceGuard g(det->device);
    if (!g.ok())
        return RADIO_EDEVICE;
    rc = enqueue_deposit_noalloc(det, chunk, (hipStream_t)stream);
    if (rc == RADIO_OK)
        det->chunks += 1;
    return rc;
}

int radio_noalloc_scratch_bytes(int64_t* bytes)
{
    if (!bytes)
        return RADIO_EINVAL;
    *bytes = (int64_t)kScratchBytes;
    return RADIO_OK;
}

int radio_deposit_batch(radio_detector* const* dets, const radio_chunk* chunks, int n,
                        void* stream)
{
    if (n < 0 || (n > 0 && (!dets || !chunks)))
        return RADIO_EINVAL;
    if (n == 0)
        return RADIO_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return RADIO_EDEVICE;
    for (int i = 0; i < n; ++i) {
        if (!dets[i])
            return RADIO_EINVAL;
        if (dets[i]->device != dev)
            return RADIO_ESTATE;
        int rc = validate_chunk(&chunks[i]);
        if (rc != RADIO_OK)
            return rc;
        if (chunks[i].n_particles > INT32_MAX || chunks[i].n_steps > INT32_MAX - 1)
            return RADIO_EINVAL;
    }
    return enqueue_batch(dets, chunks, n, (hipStream_t)stream, dev);
}

int radio_set_tuning(const radio_tuning* t)
{
    if (!t || t->target_blocks < 0 || t->target_blocks > (1 << 24) || t->items_per_workgroup < 1 ||
        t->items_per_workgroup > 4096 || t->max_grid < 1 || t->max_grid > (1 << 22) ||
        t->order_budget_mib < 0 || t->shape < 0 || t->shape >= radio::kShapes)
        return RADIO_EINVAL;
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    g_tuning = *t;
    return RADIO_OK;
}

int radio_get_tuning(radio_tuning* t)
{
    if (!t)
        return RADIO_EINVAL;
    *t = current_tuning();
    return RADIO_OK;
}

int radio_read_detector(const radio_detector* det, double* E, double* B, void* stream)
{
    if (!det)
        return RADIO_EINVAL;
    if (!E && !B)
        return RADIO_OK;
    DeviceGuard g(det->device);
    if (!g.ok())
        return RADIO_EDEVICE;
    if (radio::launch_readout(det->d_acc, det->n_c, det->n_t, det->d_user_index,
                              det->precision == RADIO_MIXED_TWOSUM, E, B,
                              (hipStream_t)stream) != hipSuccess)
        return RADIO_EDEVICE;
    return RADIO_OK;
}

int radio_detector_load(radio_detector* det, const double* E, const double* B, void* stream)
{
    if (!det || !E || !B)
        return RADIO_EINVAL;
    DeviceGuard g(det->device);
    if (!g.ok())
        return RADIO_EDEVICE;
    if (radio::launch_load(det->d_acc, det->n_c, det->n_t, det->d_user_index,
                           det->precision == RADIO_MIXED_TWOSUM, E, B,
                           (hipStream_t)stream) != hipSuccess)
        return RADIO_EDEVICE;
    return RADIO_OK;
}

int radio_detector_stats(const radio_detector* det, radio_stats* out)
{
    if (!det || !out)
        return RADIO_EINVAL;
    DeviceGuard g(det->device);
    if (!g.ok())
        return RADIO_EDEVICE;
    unsigned long long cnt[radio::kCounters] = {0, 0, 0, 0};
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(cnt, det->d_counters, sizeof(cnt), hipMemcpyDeviceToHost) != hipSuccess)
        return RADIO_EDEVICE;
    out->interactions = det->interactions;
    out->clipped = (int64_t)cnt[0];
    out->nonmonotone = (int64_t)cnt[1];
    out->bypassed = (int64_t)cnt[2];
    out->large_ring = (int64_t)cnt[3];
    out->chunks = det->chunks;
    out->slices = det->slices;
    out->bytes = (int64_t)(det->n_c * det->n_t * 6 * (int64_t)sizeof(double) +
                           det->n_c * 3 * (int64_t)sizeof(double) +
                           det->n_c * (int64_t)sizeof(int64_t) +
                           radio::kCounters * (int64_t)sizeof(unsigned long long) +
                           (int64_t)det->recs_cap +
                           (int64_t)(det->perm_cap * sizeof(int32_t)) + (int64_t)det->sel_cap);
    return RADIO_OK;
}

int radio_detector_shape(const radio_detector* det, int64_t* n_cells, int64_t* n_t,
                         int32_t* precision)
{
    if (!det)
        return RADIO_EINVAL;
    if (n_cells)
        *n_cells = det->n_c;
    if (n_t)
        *n_t = det->n_t;
    if (precision)
        *precision = det->precision;
    return RADIO_OK;
}

int radio_detector_cells(const radio_detector* det, double* out)
{
    if (!det || !out)
        return RADIO_EINVAL;
    std::memcpy(out, det->h_cells.data(), det->h_cells.size() * sizeof(double));
    return RADIO_OK;
}

int radio_arrival_times(const double* cells, const double* points, const double* t, int64_t n,
                        double c, double* out, void* stream)
{
    if (n < 0 || !std::isfinite(c) || !(c > 0.0))
        return RADIO_EINVAL;
    if (n == 0)
        return RADIO_OK;
    if (!cells || !points || !t || !out)
        return RADIO_EINVAL;
    if (radio::launch_arrival(cells, points, t, n, 1.0 / c, out, (hipStream_t)stream) !=
        hipSuccess)
        return RADIO_EDEVICE;
    return RADIO_OK;
}

int radio_slot_coordinates(const double* cells, const double* points, const double* t, int64_t n,
                           double c, double t0, double dt_det, double* out, void* stream)
{
    if (n < 0 || !std::isfinite(c) || !(c > 0.0) || !std::isfinite(t0) ||
        !std::isfinite(dt_det) || !(dt_det > 0.0) || !std::isfinite(1.0 / dt_det))
        return RADIO_EINVAL;
    if (n == 0)
        return RADIO_OK;
    if (!cells || !points || !t || !out)
        return RADIO_EINVAL;
    if (radio::launch_slot_coords(cells, points, t, n, 1.0 / c, t0, dt_det, 1.0 / dt_det,
                                  !radio::slot_quotient_corrects(dt_det), out,
                                  (hipStream_t)stream) != hipSuccess)
        return RADIO_EDEVICE;
    return RADIO_OK;
}

int radio_push(const radio_push_desc* d, int64_t n_particles, int64_t n_steps, double t_first,
               int64_t first_step, double* x, double* u, void* stream)
{
    if (!d || n_particles < 0 || n_steps < 0 || first_step < 0 || !std::isfinite(t_first) ||
        !std::isfinite(d->qm) || !std::isfinite(d->dt) || !(d->dt > 0.0) ||
        !std::isfinite(d->wave_amplitude) || !std::isfinite(d->wave_omega) ||
        !std::isfinite(d->wave_phase))
        return RADIO_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(d->E[k]) || !std::isfinite(d->B[k]) || !std::isfinite(d->wave_dir[k]) ||
            !std::isfinite(d->wave_pol[k]))
            return RADIO_EINVAL;
    if (n_particles == 0 || n_steps == 0)
        return RADIO_OK;
    if (!x || !u || n_particles > INT32_MAX || n_steps > INT32_MAX - 1)
        return RADIO_EINVAL;
    radio::PushParams P;
    P.qm = d->qm;
    P.dt = d->dt;
    for (int k = 0; k < 3; ++k) {
        P.E[k] = d->E[k];
        P.B[k] = d->B[k];
        P.wave_dir[k] = d->wave_dir[k];
        P.wave_pol[k] = d->wave_pol[k];
    }
    P.wave_amplitude = d->wave_amplitude;
    P.wave_omega = d->wave_omega;
    P.wave_phase = d->wave_phase;
    if (radio::launch_push(P, n_particles, n_steps, t_first, first_step, x, u,
                           (hipStream_t)stream) != hipSuccess)
        return RADIO_EDEVICE;
    return RADIO_OK;
}

int radio_spectrum(radio_detector* det, int64_t n_fft, const double* weights, double* d2I,
                   double* dIdw, double* dIdO, void* stream)
{
    if (!det || (!d2I && !dIdw && !dIdO))
        return RADIO_EINVAL;
    int64_t N = n_fft;
    if (N == 0) {
        N = 1;
        while (N < det->n_t)
            N *= 2;
    }
    if (N < det->n_t || N > ((int64_t)1 << 30) || (N & (N - 1)) != 0)
        return RADIO_EINVAL;
    DeviceGuard g(det->device);
    if (!g.ok())
        return RADIO_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    const bool pairs = det->precision == RADIO_MIXED_TWOSUM;
    // cells per group: two complex work arrays of 2 G N values within ~1 GiB
    const int64_t per_cell = 2 * 2 * N * (int64_t)sizeof(double2);
    const int64_t G = std::max<int64_t>(1, std::min<int64_t>(det->n_c, ((int64_t)1 << 30) / per_cell));
    double2* w0 = nullptr;
    double2* w1 = nullptr;
    double* d_w = nullptr;
    int rc = RADIO_OK;
    if (d2I || dIdw) {
        // the two work arrays, kept by the detector for later spectra
        rc = grow(&det->d_spec, &det->spec_cap, (size_t)(4 * G * N + radio::kSpecTableValues), s);
        w0 = det->d_spec;
        w1 = det->d_spec + 2 * G * N;
    }
    if (rc == RADIO_OK && weights && dIdw) {
        if (hipMalloc((void**)&d_w, (size_t)det->n_c * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            rc = RADIO_ENOMEM;
        } else if (hipMemcpyAsync(d_w, weights, (size_t)det->n_c * sizeof(double),
                                  hipMemcpyHostToDevice, s) != hipSuccess) {
            rc = RADIO_EDEVICE;
        }
    }
    bool parseval_done = false;  // every group computed its cells' dI/dOmega on the way
    if (rc == RADIO_OK && (d2I || dIdw)) {
        parseval_done = true;
        for (int64_t r0 = 0; r0 < det->n_c && rc == RADIO_OK; r0 += G) {
            const int64_t Gi = std::min(G, det->n_c - r0);
            bool done = false;
            if (radio::launch_spectrum_group(det->d_acc, pairs, det->n_t, r0, Gi, N, det->d_cells,
                                             det->d_user_index, d_w, det->dt_det, det->c, w0, w1,
                                             det->d_spec + 4 * G * N, d2I, dIdw, dIdO, &done,
                                             r0 == 0, s) != hipSuccess)
                rc = RADIO_EDEVICE;
            parseval_done = parseval_done && done;
        }
    }
    if (rc == RADIO_OK && dIdO && !parseval_done &&
        radio::launch_spectrum_parseval(det->d_acc, pairs, det->n_c, det->n_t, det->d_cells,
                                        det->d_user_index, det->dt_det, det->c, dIdO,
                                        s) != hipSuccess)
        rc = RADIO_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess && rc == RADIO_OK)
        rc = RADIO_EDEVICE;
    if (d_w)
        (void)hipFree(d_w);
    return rc;
}

}  // extern "C"
