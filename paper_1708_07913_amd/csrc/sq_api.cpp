// Host side of libsq: the C ABI of include/sq.h.
//
// Argument validation, the per-atom projector tables (z-runs of the sphere
// of radius r_c, Sec. 3.1 trapezoid normalisation), the coefficient table of
// the discrete-orthogonality rule (Sec. 3.2), workspace layout, kernel
// launches and Brent's method for the Fermi level (Sec. 3.2) around the
// device-side electron count.  Compiled without floating-point contraction so
// that the sphere membership test r^2 <= r_c^2 is evaluated exactly as
// written.
#include "../../include/sq.h"
#include "sq_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <new>
#include <string>
#include <vector>

namespace {

thread_local std::string g_error;

int fail(int code, const std::string &msg) {
    g_error = msg;
    return code;
}

bool is_finite(double v) { return std::isfinite(v); }

enum State { kSetup = 0, kBound = 1, kBounds = 2 };

constexpr int kReduceBlocks = 1024;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

uint64_t splitmix64_first(uint64_t seed) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

}  // namespace

struct sq_ctx {
    double cell = 0, h = 0, kT = 0;
    int n = 0, fd_order = 0, no = 0, m = 0, C = 0, npl = 0, nq = 0;
    long long nd = 0, ns = 0;
    sq_options opt{};
    double w[sq::kNoMax + 1] = {0};
    std::vector<sq::AtomDev> atoms;
    std::vector<sq::RunDev> runs;
    std::vector<double> pvals;
    std::vector<double> ctab, rk;
    double start_norm = 0;
    int device = 0;
    int nwg_lanczos = 0, nwg_moments = 0, nwg_slots = 0;
    int nch = 2;        // projector chains per cube column (max sphere overlap depth)
    int pstride = 0;    // doubles between a projector value and the one a plane above
    int max_overlap = 0;
    size_t off_atoms = 0, off_runs = 0, off_pvals = 0, off_chi = 0, off_zeta = 0, off_ctab = 0,
           off_rk = 0, off_W = 0, off_part = 0, off_scal = 0, off_flags = 0, off_forces = 0,
           off_slots = 0, off_wslots = 0, off_xslots = 0, off_args = 0, total = 0;
    sq::RecurrenceArgs args_host[2] = {};  // staged launch arguments (Lanczos, moments)
    char *ws = nullptr;
    const double *veff = nullptr;
    int state = kSetup;
    // bumped whenever chi/zeta are rewritten (sq_spectral_bounds, sq_set_bounds,
    // a batched pass with bounds), so a batch can tell whether the bounds it
    // would reuse are still its own
    unsigned long long bounds_gen = 0;

    template <typename T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

namespace {

// Central FD weights of order 2 n_o (Sec. 3.1):
//   w_0 = -(1/h^2) sum_{q<=n_o} 1/q^2,
//   w_d = 2 (-1)^{d+1} / (h^2 d^2) * (n_o!)^2 / ((n_o - d)! (n_o + d)!).
void laplacian_weights(int no, double h, double *w) {
    double s = 0.0;
    for (int q = 1; q <= no; ++q) s += 1.0 / (double(q) * q);
    w[0] = -s / (h * h);
    // (n_o!)^2 / ((n_o-d)! (n_o+d)!) = prod_{i=1..d} (n_o - d + i) / (n_o + i)
    for (int d = 1; d <= sq::kNoMax; ++d) {
        if (d > no) {
            w[d] = 0.0;
            continue;
        }
        double ratio = 1.0;
        for (int i = 1; i <= d; ++i) ratio *= double(no - d + i) / double(no + i);
        const double sign = (d & 1) ? 1.0 : -1.0;
        w[d] = 2.0 * sign * ratio / (h * h * double(d) * d);
    }
}

// Reach of an atom's projector sphere in grid steps from its base node: the
// sphere's points have offsets -r .. r + 1 in each direction.
int sphere_reach(double rc, double h) { return int(std::ceil(rc / h)) + 1; }

// Central first-derivative weights of order 2 n_o (Sec. 3.1 gradient):
// gw_d = (-1)^{d+1} / (h d) (n_o!)^2 / ((n_o - d)! (n_o + d)!).
void gradient_weights(int no, double h, double *gw) {
    gw[0] = 0.0;
    for (int d = 1; d <= sq::kNoMax; ++d) {
        if (d > no) {
            gw[d] = 0.0;
            continue;
        }
        double ratio = 1.0;
        for (int i = 1; i <= d; ++i) ratio *= double(no - d + i) / double(no + i);
        const double sign = (d & 1) ? 1.0 : -1.0;
        gw[d] = sign * ratio / (h * double(d));
    }
}

// Projector of one atom as z-runs over (dx, dy) columns of its sphere.  The
// values sit in a box of (2 rbox + 2)^3 doubles, x fastest and zero outside
// the sphere, so that neighbouring columns of one plane are neighbours in
// memory (a wave's loads of one plane coalesce); a run's value at the next
// plane is c->pstride doubles further.
int build_atom_table(sq_ctx *c, const double *R, double sig, double rc, double gamma, int rbox) {
    const double h = c->h;
    const int b[3] = {int(std::floor(R[0] / h)), int(std::floor(R[1] / h)), int(std::floor(R[2] / h))};
    const int r = sphere_reach(rc, h);
    const double rc2 = rc * rc;
    const int W = 2 * rbox + 2;
    if (size_t(c->pvals.size()) + size_t(W) * W * W > size_t(std::numeric_limits<int32_t>::max() / 2))
        return fail(SQ_EINVAL, "projector tables too large");
    sq::AtomDev at{};
    at.bx = b[0];
    at.by = b[1];
    at.bz = b[2];
    at.run0 = int(c->runs.size());
    for (int k = 0; k < 3; ++k) {
        at.dmin[k] = std::numeric_limits<int>::max();
        at.dmax[k] = std::numeric_limits<int>::min();
    }
    const size_t v0 = c->pvals.size();
    c->pvals.resize(v0 + size_t(W) * W * W, 0.0);
    auto box = [&](int dx, int dy, int dz) {
        return v0 + (size_t(dz + rbox) * W + size_t(dy + rbox)) * W + size_t(dx + rbox);
    };
    double ss = 0.0;  // sum of squares, in the order of the scan
    for (int dy = -r; dy <= r + 1; ++dy) {
        for (int dx = -r; dx <= r + 1; ++dx) {
            int first = 0, count = 0;
            for (int dz = -r; dz <= r + 1; ++dz) {
                const double ex = double(b[0] + dx) * h - R[0];
                const double ey = double(b[1] + dy) * h - R[1];
                const double ez = double(b[2] + dz) * h - R[2];
                const double r2 = ex * ex + ey * ey + ez * ez;
                if (r2 <= rc2) {
                    if (count > 0 && dz != first + count)
                        return fail(SQ_EINVAL, "projector sphere column is not contiguous");
                    if (count == 0) first = dz;
                    ++count;
                    const double v = std::exp(-r2 / (2.0 * sig * sig));
                    c->pvals[box(dx, dy, dz)] = v;
                    ss += v * v;
                }
            }
            if (count == 0) continue;
            if (count > 255) return fail(SQ_EINVAL, "projector radius too large for the mesh");
            sq::RunDev run{};
            run.dx = int8_t(dx);
            run.dy = int8_t(dy);
            run.dz0 = int8_t(first);
            run.len = uint8_t(count);
            run.vstart = int32_t(box(dx, dy, first));
            c->runs.push_back(run);
            const int lo[3] = {dx, dy, first}, hi[3] = {dx, dy, first + count - 1};
            for (int k = 0; k < 3; ++k) {
                at.dmin[k] = std::min(at.dmin[k], lo[k]);
                at.dmax[k] = std::max(at.dmax[k], hi[k]);
            }
        }
    }
    at.nrun = int(c->runs.size()) - at.run0;
    if (at.nrun == 0) {
        for (int k = 0; k < 3; ++k) at.dmin[k] = at.dmax[k] = 0;
    }
    // normalise on the grid: h^3 sum chi^2 = 1 over the whole sphere (the
    // box's zeros stay zero)
    const double norm = std::sqrt(h * h * h * ss);
    for (size_t i = v0; i < c->pvals.size(); ++i) c->pvals[i] /= norm;
    at.coef = gamma * h * h * h;
    c->atoms.push_back(at);
    return SQ_OK;
}

int hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return SQ_OK;
    return fail(SQ_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int flags_status(int flags) {
    if (flags & sq::kFlagImages) return fail(SQ_ECAPACITY, "more projector images in a region than supported");
    if (flags & sq::kFlagRuns) return fail(SQ_ECAPACITY, "projector run table of a region overflowed");
    if (flags & sq::kFlagOverlap) return fail(SQ_ECAPACITY, "more than two projector spheres overlap");
    if (flags & sq::kFlagLanczos) return fail(SQ_EINVAL, "non-finite Lanczos coefficient (check V_eff)");
    if (flags & sq::kFlagBounds) return fail(SQ_EBOUNDS, "a Chebyshev moment left [-1, 1]: bounds too tight");
    return SQ_OK;
}

int read_flags(sq_ctx *c, hipStream_t s) {
    int flags = 0;
    int rc = hip_check(hipMemcpyAsync(&flags, c->at<int>(c->off_flags), sizeof(int), hipMemcpyDeviceToHost, s),
                       "reading device flags");
    if (rc) return rc;
    rc = hip_check(hipStreamSynchronize(s), "kernel execution");
    if (rc) return rc;
    return flags_status(flags);
}

sq::RecurrenceArgs recurrence_args(sq_ctx *c) {
    sq::RecurrenceArgs a{};
    a.n = c->n;
    a.m = c->m;
    a.C = c->C;
    a.nd = c->nd;
    for (int d = 0; d <= sq::kNoMax; ++d) a.w[d] = c->w[d];
    a.veff = c->veff;
    a.natom = int(c->atoms.size());
    a.atoms = c->at<sq::AtomDev>(c->off_atoms);
    a.runs = c->at<sq::RunDev>(c->off_runs);
    a.pvals = c->at<double>(c->off_pvals);
    a.pvals_bytes = (long long)(c->pvals.size() * sizeof(double));
    a.pstride = c->pstride;
    a.chi = c->at<double>(c->off_chi);
    a.zeta = c->at<double>(c->off_zeta);
    a.npl = c->npl;
    a.flags = c->at<int>(c->off_flags);
    a.nch = c->nch;
    a.n_lanczos = c->opt.n_lanczos;
    a.start_norm = c->start_norm;
    a.margin = c->opt.margin;
    a.bounds_tol = c->opt.precision == SQ_FP32_MIXED ? 1e-5 : 1e-10;
    gradient_weights(c->no, c->h, a.gw);
    a.ctab = c->at<double>(c->off_ctab);
    a.rk = c->at<double>(c->off_rk);
    a.kT = c->kT;
    return a;
}

// Stage the arguments of one recurrence launch in the workspace (kernels read
// them from device memory) and describe the launch: every node of this
// snapshot, split statically over the XCDs.
int stage_launch(sq_ctx *c, const sq::RecurrenceArgs &a, int which, hipStream_t s, sq::LaunchArgs *k) {
    c->args_host[which] = a;
    sq::RecurrenceArgs *dev = c->at<sq::RecurrenceArgs>(c->off_args) + which;
    int rc = hip_check(hipMemcpyAsync(dev, &c->args_host[which], sizeof(a), hipMemcpyHostToDevice, s),
                       "staging launch arguments");
    if (rc) return rc;
    *k = sq::LaunchArgs{};
    k->snaps = dev;
    k->slots = c->ws + c->off_slots;
    k->wslots = c->ws + c->off_wslots;
    k->xslots = c->ws + c->off_xslots;
    k->slot_elems = sq::slot_elems_for(c->C);
    return SQ_OK;
}

int pick_workgroups(sq_ctx *c) {
    int dev = 0;
    int rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (rc) return rc;
    c->device = dev;
    int cus = 0;
    rc = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
    if (rc) return rc;
    const bool mixed = c->opt.precision == SQ_FP32_MIXED;
    int bl = 0, bm = 0;
    rc = hip_check(sq::recurrence_occupancy(c->C, true, false, c->nch, &bl), "occupancy (Lanczos)");
    if (rc) return rc;
    rc = hip_check(sq::recurrence_occupancy(c->C, false, mixed, c->nch, &bm), "occupancy (moments)");
    if (rc) return rc;
    if (bl < 1 || bm < 1) return fail(SQ_EDEVICE, "recurrence kernel does not fit on a compute unit");
    auto round8 = [](long long v) { return int(std::max<long long>(8, (v + 7) / 8 * 8)); };
    const long long cap = (c->nd + 7) / 8 * 8;
    if (c->opt.workgroups > 0) {
        c->nwg_lanczos = c->nwg_moments = round8(c->opt.workgroups);
    } else {
        c->nwg_lanczos = round8(std::min<long long>(cap, (long long)cus * bl / 8 * 8));
        c->nwg_moments = round8(std::min<long long>(cap, (long long)cus * bm / 8 * 8));
    }
    c->nwg_slots = std::max(c->nwg_lanczos, c->nwg_moments);
    return SQ_OK;
}

void layout(sq_ctx *c) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + std::max<size_t>(bytes, 1));
        return o;
    };
    c->off_atoms = take(c->atoms.size() * sizeof(sq::AtomDev));
    c->off_runs = take(c->runs.size() * sizeof(sq::RunDev));
    c->off_pvals = take(c->pvals.size() * sizeof(double));
    c->off_chi = take(size_t(c->nd) * sizeof(double));
    c->off_zeta = take(size_t(c->nd) * sizeof(double));
    c->off_ctab = take(c->ctab.size() * sizeof(double));
    c->off_rk = take(c->rk.size() * sizeof(double));
    c->off_W = take(size_t(c->nd) * c->nq * sizeof(double));
    c->off_part = take(3 * kReduceBlocks * sizeof(double));
    c->off_scal = take(8 * sizeof(double));
    c->off_flags = take(64);
    c->off_forces = take(c->atoms.size() * 3 * sizeof(double));
    c->off_args = take(2 * sizeof(sq::RecurrenceArgs));
    // one slot per workgroup: C planes of slot_plane(C) doubles
    const size_t se = size_t(sq::slot_elems_for(c->C));
    c->off_slots = take(size_t(c->nwg_slots) * se * sizeof(double));
    // streamed regions (wider than kResidentCube) need a second buffer in the
    // moments sweep and a third in Lanczos
    const bool stream = c->C > sq::kResidentCube;
    c->off_wslots = take(size_t(stream ? c->nwg_slots : c->nwg_lanczos) * se * sizeof(double));
    c->off_xslots = take(stream ? size_t(c->nwg_lanczos) * se * sizeof(double) : 0);
    c->total = off;
}

int upload_veff(sq_ctx *c, const double *veff, hipStream_t) {
    c->veff = veff;  // read in FP64 by every kernel (the mixed one included)
    return SQ_OK;
}

int device_scalars(sq_ctx *c, hipStream_t s, double *out, int count) {
    int rc = hip_check(hipMemcpyAsync(out, c->at<double>(c->off_scal), sizeof(double) * count,
                                      hipMemcpyDeviceToHost, s), "reading device scalars");
    if (rc) return rc;
    return hip_check(hipStreamSynchronize(s), "reduction");
}

int electron_count(sq_ctx *c, double mu, hipStream_t s, double *out) {
    int rc = hip_check(sq::launch_count(c->at<double>(c->off_W), c->at<double>(c->off_chi),
                                        c->at<double>(c->off_zeta), c->at<double>(c->off_rk), c->nd, c->nq, mu,
                                        c->kT, c->at<double>(c->off_part), kReduceBlocks,
                                        c->at<double>(c->off_scal), s),
                       "electron count");
    if (rc) return rc;
    double v = 0;
    rc = device_scalars(c, s, &v, 1);
    if (rc) return rc;
    *out = 2.0 * v;
    return SQ_OK;
}

int check_ctx(const sq_ctx *c, int need) {
    if (!c) return fail(SQ_EINVAL, "null context");
    if (c->state < need) {
        static const char *names[] = {"sq_setup", "sq_bind", "sq_spectral_bounds or sq_set_bounds"};
        return fail(SQ_ESTATE, std::string("call order: ") + names[need] + " has not been called");
    }
    return SQ_OK;
}

template <typename F>
int guarded(F f) {
    try {
        return f();
    } catch (const std::bad_alloc &) {
        return fail(SQ_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(SQ_EINVAL, "unexpected host exception");
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Batched snapshots
// ---------------------------------------------------------------------------
static_assert(SQ_SHAPE_TWO_ROWS == sq::kShapeTwoRows && SQ_SHAPE_TWO_PLANES == sq::kShapeTwoPlanes,
              "public and internal kernel shape bits");

struct sq_batch {
    struct Group {
        int C = 0, nch = 2;
        std::vector<int> snaps;
        int shape = 0;              // kernel shape bits (sq::kShape*) of this group's launches
        int occ_l = 1, occ_m = 1;   // resident workgroups per CU (Lanczos, moments) at that shape
        int occ_lv[4] = {0, 0, 0, 0}, occ_mv[4] = {0, 0, 0, 0};  // the same for every shape the cube has
        int item0 = 0, n_items = 0; // range in the item table
        void set_shape(int sh) {
            shape = sh;
            occ_l = occ_lv[sh];
            occ_m = occ_mv[sh];
        }
    };
    std::vector<sq_ctx *> ctx;
    std::vector<double *> moments, rho;
    std::vector<double> n_e;
    sq_batch_options opt{};
    bool mixed = false;
    int device = 0, cus = 0, max_brent = 200;
    char device_name[256] = {0};
    std::vector<Group> groups;
    long long max_slot = 0;          // largest workgroup slot (doubles) of any snapshot and shape
    int nwg_cap = 0;                 // largest grid of any launch (buffers are sized for it)
    int block_nodes = 32, wg_per_cu = 0;
    std::vector<sq::WorkItem> items;
    std::vector<sq::RecurrenceArgs> args;
    std::vector<sq::FermiSnap> fermi;
    std::vector<sq::BrentParams> prm;
    std::vector<sq::BrentState> state_host;
    std::vector<double> scal_host;
    std::vector<int> flags_host;
    size_t off_args = 0, off_items = 0, off_counters = 0, off_fermi = 0, off_prm = 0, off_state = 0, off_ext = 0,
           off_part = 0, off_slots = 0, off_wslots = 0, off_xslots = 0, total = 0;
    size_t items_capacity = 0;
    char *ws = nullptr;
    hipStream_t own = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};       // [0]: bounds reused, [1]: with bounds
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    long long passes = 0;
    bool have_bounds = false;
    std::vector<double> slack;       // per snapshot: min_q zeta_q margin / (1 + margin) of the last bounds
    std::vector<unsigned long long> gen_seen;  // per snapshot: bounds generation after the last batched pass
    size_t off_vref = 0, off_red = 0;  // V_eff at the last bounds; reduction outputs (2 per snapshot)

    template <typename T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    ~sq_batch() {
        for (int i = 0; i < 2; ++i) {
            if (exec[i]) (void)hipGraphExecDestroy(exec[i]);
            if (graph[i]) (void)hipGraphDestroy(graph[i]);
        }
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (own) (void)hipStreamDestroy(own);
    }
};

namespace {

void drop_graph(sq_batch *b) {
    for (int i = 0; i < 2; ++i) {
        if (b->exec[i]) (void)hipGraphExecDestroy(b->exec[i]);
        if (b->graph[i]) (void)hipGraphDestroy(b->graph[i]);
        b->exec[i] = nullptr;
        b->graph[i] = nullptr;
    }
}

int batch_grid(const sq_batch *b, const sq_batch::Group &g, bool lanczos) {
    const int occ = lanczos ? g.occ_l : g.occ_m;
    const int per_cu = b->wg_per_cu > 0 ? std::min(b->wg_per_cu, occ) : occ;
    return std::max(1, std::min(g.n_items, b->cus * per_cu));
}

// Work items: blocks of block_nodes consecutive nodes of the first
// `fraction` of every snapshot's nodes; per group, the most expensive
// snapshots (per-node cost ~ N_s (n_lanczos + n_pl / 2)) first.
void build_items(sq_batch *b, int block_nodes, double fraction) {
    b->items.clear();
    for (auto &g : b->groups) {
        g.item0 = int(b->items.size());
        std::vector<int> order = g.snaps;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            const sq_ctx *a = b->ctx[size_t(x)], *c = b->ctx[size_t(y)];
            return a->opt.n_lanczos * 2 + a->npl > c->opt.n_lanczos * 2 + c->npl;
        });
        for (int si : order) {
            const sq_ctx *c = b->ctx[size_t(si)];
            const long long nodes = std::max<long long>(1, (long long)std::ceil(double(c->nd) * fraction));
            for (long long q = 0; q < std::min(nodes, c->nd); q += block_nodes) {
                sq::WorkItem it{};
                it.snap = si;
                it.q0 = q;
                it.q1 = std::min({q + block_nodes, nodes, c->nd});
                b->items.push_back(it);
            }
        }
        g.n_items = int(b->items.size()) - g.item0;
    }
}

int upload_items(sq_batch *b, hipStream_t s) {
    if (b->items.size() > b->items_capacity) return fail(SQ_ENOMEM, "work-item table larger than its workspace region");
    return hip_check(hipMemcpyAsync(b->at<sq::WorkItem>(b->off_items), b->items.data(),
                                    b->items.size() * sizeof(sq::WorkItem), hipMemcpyHostToDevice, s),
                     "uploading work items");
}

// Snapshot arguments are re-staged before every pass: V_eff may have been
// replaced (sq_update_veff) since the previous one.
int upload_args(sq_batch *b, hipStream_t s) {
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        b->args[i] = recurrence_args(b->ctx[i]);
        b->args[i].moments = b->moments[i];
    }
    return hip_check(hipMemcpyAsync(b->at<sq::RecurrenceArgs>(b->off_args), b->args.data(),
                                    b->args.size() * sizeof(sq::RecurrenceArgs), hipMemcpyHostToDevice, s),
                     "staging snapshot arguments");
}

sq::LaunchArgs group_launch(sq_batch *b, const sq_batch::Group &g, int counter) {
    sq::LaunchArgs k{};
    k.snaps = b->at<sq::RecurrenceArgs>(b->off_args);
    k.items = b->at<sq::WorkItem>(b->off_items) + g.item0;
    k.n_items = g.n_items;
    k.counter = b->at<int>(b->off_counters) + counter;
    k.slots = b->ws + b->off_slots;
    k.wslots = b->ws + b->off_wslots;
    k.xslots = b->ws + b->off_xslots;
    k.slot_elems = b->max_slot;
    return k;
}

// only >= 0: launch that group alone (the autotuner's per-group timing)
int enqueue_recurrences(sq_batch *b, bool lanczos, bool moments, hipStream_t s, int only = -1) {
    const int ng = int(b->groups.size());
    int rc = hip_check(sq::launch_zero_ints(b->at<int>(b->off_counters), 2 * ng, s), "clearing work queues");
    if (rc) return rc;
    for (sq_ctx *c : b->ctx) {
        rc = hip_check(sq::launch_zero_ints(c->at<int>(c->off_flags), 1, s), "clearing flags");
        if (rc) return rc;
    }
    for (int gi = 0; lanczos && gi < ng; ++gi) {
        const auto &g = b->groups[size_t(gi)];
        if (g.n_items == 0 || (only >= 0 && gi != only)) continue;
        rc = hip_check(
            sq::launch_lanczos(group_launch(b, g, 2 * gi), g.C, g.nch, batch_grid(b, g, true), s, g.shape),
            "launching batched Lanczos");
        if (rc) return rc;
    }
    for (int gi = 0; moments && gi < ng; ++gi) {
        const auto &g = b->groups[size_t(gi)];
        if (g.n_items == 0 || (only >= 0 && gi != only)) continue;
        rc = hip_check(sq::launch_moments(group_launch(b, g, 2 * gi + 1), g.C, g.nch, b->mixed,
                                          batch_grid(b, g, false), s, g.shape),
                       "launching batched moments");
        if (rc) return rc;
    }
    return SQ_OK;
}

// The whole pass, without host round trips (so that it can be captured).
int enqueue_pass(sq_batch *b, bool bounds, hipStream_t s) {
    int rc = enqueue_recurrences(b, bounds, true, s);
    if (rc) return rc;
    const int n = int(b->ctx.size());
    for (int i = 0; i < n; ++i) {
        sq_ctx *c = b->ctx[size_t(i)];
        rc = hip_check(sq::launch_quadrature_weights(b->moments[size_t(i)], c->at<double>(c->off_ctab),
                                                     c->at<double>(c->off_W), c->nd, c->npl, s),
                       "quadrature weights");
        if (rc) return rc;
        rc = hip_check(sq::launch_extent(c->at<double>(c->off_chi), c->at<double>(c->off_zeta), c->nd,
                                         c->at<double>(c->off_part), kReduceBlocks, b->at<double>(b->off_ext) + 2 * i,
                                         s),
                       "spectral extent");
        if (rc) return rc;
    }
    sq::BrentState *st = b->at<sq::BrentState>(b->off_state);
    rc = hip_check(sq::launch_brent_begin(st, b->at<sq::BrentParams>(b->off_prm), b->at<double>(b->off_ext), n, s),
                   "Fermi level");
    if (rc) return rc;
    // two bracket evaluations, then at most max_brent iterations
    for (int it = 0; it < b->max_brent + 2; ++it) {
        rc = hip_check(sq::launch_count_batch(b->at<sq::FermiSnap>(b->off_fermi), st, n, b->at<double>(b->off_part),
                                              kReduceBlocks, s),
                       "electron count");
        if (rc) return rc;
        rc = hip_check(sq::launch_brent_feed(st, b->at<double>(b->off_part), kReduceBlocks, n, s), "Brent step");
        if (rc) return rc;
    }
    for (int i = 0; i < n; ++i) {
        sq_ctx *c = b->ctx[size_t(i)];
        const double h3 = c->h * c->h * c->h;
        rc = hip_check(sq::launch_density(c->at<double>(c->off_W), c->at<double>(c->off_chi),
                                          c->at<double>(c->off_zeta), c->at<double>(c->off_rk), c->nd, c->nq, 0.0,
                                          &st[i].xb, c->kT, h3, b->rho[size_t(i)], c->at<double>(c->off_part),
                                          kReduceBlocks, c->at<double>(c->off_scal), s),
                       "density");
        if (rc) return rc;
    }
    return SQ_OK;
}

// Collect the per-snapshot results of a pass (after it was enqueued on s).
int finish_pass(sq_batch *b, hipStream_t s, double *mu, double *energies) {
    const size_t n = b->ctx.size();
    int rc = hip_check(hipMemcpyAsync(b->state_host.data(), b->at<sq::BrentState>(b->off_state),
                                      n * sizeof(sq::BrentState), hipMemcpyDeviceToHost, s),
                       "reading Fermi levels");
    for (size_t i = 0; !rc && i < n; ++i) {
        sq_ctx *c = b->ctx[i];
        rc = hip_check(hipMemcpyAsync(&b->scal_host[3 * i], c->at<double>(c->off_scal), 3 * sizeof(double),
                                      hipMemcpyDeviceToHost, s),
                       "reading energies");
        if (!rc)
            rc = hip_check(hipMemcpyAsync(&b->flags_host[i], c->at<int>(c->off_flags), sizeof(int),
                                          hipMemcpyDeviceToHost, s),
                           "reading device flags");
    }
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "batched pass");
    if (rc) return rc;
    int first = SQ_OK;
    std::string msg;
    for (size_t i = 0; i < n; ++i) {
        sq_ctx *c = b->ctx[i];
        int st = flags_status(b->flags_host[i]);
        const sq::BrentState &bs = b->state_host[i];
        if (!st && bs.phase != sq::kBrentDone) {
            st = fail(SQ_ENOCONV, bs.phase == sq::kBrentNonFinite ? "non-finite electron count"
                                  : bs.phase == sq::kBrentNoSign
                                      ? "electron count does not change sign over the spectral bracket"
                                      : "Fermi level search did not converge");
        }
        if (st) {
            if (!first) {
                first = st;
                msg = "snapshot " + std::to_string(i) + ": " + g_error;
            }
            continue;
        }
        c->state = kBounds;
        const double h3 = c->h * c->h * c->h;
        if (mu) mu[i] = bs.xb;
        if (energies) {
            energies[4 * i] = b->scal_host[3 * i];
            energies[4 * i + 1] = b->scal_host[3 * i + 1];
            energies[4 * i + 2] = b->scal_host[3 * i] + b->scal_host[3 * i + 1];
            energies[4 * i + 3] = h3 * b->scal_host[3 * i + 2];
        }
    }
    if (first) return fail(first, msg);
    return SQ_OK;
}

// Reusing bounds is safe while V_eff has moved by less than half the margin
// slack since they were computed: the potential enters H_q as a diagonal, so
// by Weyl's inequality no eigenvalue moves further than max |delta V|.
int reuse_is_safe(sq_batch *b, hipStream_t s, bool *safe) {
    const size_t n = b->ctx.size();
    double *out = b->at<double>(b->off_red);
    size_t vo = 0;
    for (size_t i = 0; i < n; ++i) {
        sq_ctx *c = b->ctx[i];
        int rc = hip_check(sq::launch_diff_extent(c->veff, b->at<double>(b->off_vref) + vo, c->nd,
                                                  b->at<double>(b->off_part), kReduceBlocks, out + 2 * i, s),
                           "potential change");
        if (rc) return rc;
        vo += size_t(c->nd);
    }
    std::vector<double> ext(2 * n);
    int rc = hip_check(hipMemcpyAsync(ext.data(), out, 2 * n * sizeof(double), hipMemcpyDeviceToHost, s),
                       "potential change");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "potential change");
    if (rc) return rc;
    *safe = true;
    for (size_t i = 0; i < n; ++i) {
        const double dv = std::max(-ext[2 * i], ext[2 * i + 1]);
        if (!(dv <= 0.5 * b->slack[i])) *safe = false;
    }
    return SQ_OK;
}

// After a pass that computed bounds: remember V_eff and the margin slack.
int record_bounds(sq_batch *b, hipStream_t s) {
    const size_t n = b->ctx.size();
    double *out = b->at<double>(b->off_red);
    size_t vo = 0;
    for (size_t i = 0; i < n; ++i) {
        sq_ctx *c = b->ctx[i];
        int rc = hip_check(hipMemcpyAsync(b->at<double>(b->off_vref) + vo, c->veff, size_t(c->nd) * sizeof(double),
                                          hipMemcpyDeviceToDevice, s),
                           "keeping V_eff");
        if (!rc)
            rc = hip_check(sq::launch_diff_extent(c->at<double>(c->off_zeta), nullptr, c->nd,
                                                  b->at<double>(b->off_part), kReduceBlocks, out + 2 * i, s),
                           "margin slack");
        if (rc) return rc;
        vo += size_t(c->nd);
    }
    std::vector<double> ext(2 * n);
    int rc = hip_check(hipMemcpyAsync(ext.data(), out, 2 * n * sizeof(double), hipMemcpyDeviceToHost, s),
                       "margin slack");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "margin slack");
    if (rc) return rc;
    b->slack.assign(n, 0.0);
    for (size_t i = 0; i < n; ++i) {
        const double m = b->ctx[i]->opt.margin;
        b->slack[i] = ext[2 * i] * m / (1.0 + m);
    }
    return SQ_OK;
}

int batch_layout(sq_batch *b) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + std::max<size_t>(bytes, 1));
        return o;
    };
    const size_t n = b->ctx.size(), ng = b->groups.size();
    // the item table must hold the smallest block size the tuner tries
    size_t cap = 0;
    for (sq_ctx *c : b->ctx) cap += size_t((c->nd + 7) / 8);
    b->items_capacity = cap;
    b->off_args = take(n * sizeof(sq::RecurrenceArgs));
    b->off_items = take(cap * sizeof(sq::WorkItem));
    b->off_counters = take(2 * ng * sizeof(int));
    b->off_fermi = take(n * sizeof(sq::FermiSnap));
    b->off_prm = take(n * sizeof(sq::BrentParams));
    b->off_state = take(n * sizeof(sq::BrentState));
    b->off_ext = take(2 * n * sizeof(double));
    b->off_part = take(std::max<size_t>(n, 2) * size_t(kReduceBlocks) * sizeof(double));
    size_t vtot = 0;
    for (sq_ctx *c : b->ctx) vtot += size_t(c->nd);
    b->off_vref = take(vtot * sizeof(double));
    b->off_red = take(2 * n * sizeof(double));
    const size_t slot = size_t(b->nwg_cap) * size_t(b->max_slot) * sizeof(double);
    bool stream = false;
    for (const auto &g : b->groups) stream = stream || g.C > sq::kResidentCube;
    b->off_slots = take(slot);
    b->off_wslots = take(slot);
    b->off_xslots = take(stream ? slot : 0);
    b->total = off;
    return SQ_OK;
}

// Autotuner cache: a flat JSON object
// {"key": {"block_nodes": B, "wg_per_cu": W, "shapes": [[C, nch, bits], ...],
//          "shape_ms": [[C, nch, t0, t1, t2, t3], ...], "ms": T}, ...}
// where t_s is the sample time (ms) of shape bits s for that group, -1 where
// its cube side lacks the shape (shape_ms is informative; lookups ignore it).
std::string tune_key(const sq_batch *b) {
    std::vector<std::string> parts;
    for (const auto &g : b->groups) {
        long long nodes = 0;
        for (int si : g.snaps) nodes += b->ctx[size_t(si)]->nd;
        parts.push_back("C" + std::to_string(g.C) + "x" + std::to_string(g.nch) + ":" + std::to_string(nodes));
    }
    std::sort(parts.begin(), parts.end());
    // "lms": timed on the Lanczos and moments launches together, with kernel shapes
    std::string key = std::string(b->device_name) + "/" + std::to_string(b->cus) + "cu/lms/" + (b->mixed ? "mixed" : "fp64");
    for (const auto &p : parts) key += "/" + p;
    return key;
}

struct TunedShape {
    int C, nch, shape;
    double ms[4];
};

bool cache_lookup(const char *path, const std::string &key, int *block, int *wg, std::vector<TunedShape> *shapes) {
    if (!path) return false;
    FILE *f = std::fopen(path, "rb");
    if (!f) return false;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    std::fclose(f);
    const size_t at = text.find("\"" + key + "\"");
    if (at == std::string::npos) return false;
    const size_t pb = text.find("\"block_nodes\":", at), pw = text.find("\"wg_per_cu\":", at);
    const size_t ps = text.find("\"shapes\":", at);
    if (pb == std::string::npos || pw == std::string::npos || ps == std::string::npos) return false;
    if (std::sscanf(text.c_str() + pb + 14, "%d", block) != 1 || std::sscanf(text.c_str() + pw + 12, "%d", wg) != 1)
        return false;
    size_t i = text.find('[', ps);
    if (i == std::string::npos) return false;
    shapes->clear();
    for (++i;;) {
        while (i < text.size() && (text[i] == ' ' || text[i] == ',' || text[i] == '\n')) ++i;
        if (i >= text.size()) return false;
        if (text[i] == ']') return true;
        TunedShape t{0, 0, 0, {-1.0, -1.0, -1.0, -1.0}};
        if (text[i] != '[' || std::sscanf(text.c_str() + i, "[%d, %d, %d]", &t.C, &t.nch, &t.shape) != 3) return false;
        shapes->push_back(t);
        i = text.find(']', i);
        if (i == std::string::npos) return false;
        ++i;
    }
}

void cache_store(const char *path, const std::string &key, int block, int wg, const std::vector<TunedShape> &shapes,
                 double ms) {
    if (!path) return;
    std::string text;
    if (FILE *f = std::fopen(path, "rb")) {
        char buf[4096];
        size_t got;
        while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
        std::fclose(f);
    }
    const size_t close = text.rfind('}');
    std::string sh = "[";
    for (size_t i = 0; i < shapes.size(); ++i)
        sh += (i ? ", [" : "[") + std::to_string(shapes[i].C) + ", " + std::to_string(shapes[i].nch) + ", " +
              std::to_string(shapes[i].shape) + "]";
    sh += "], \"shape_ms\": [";
    for (size_t i = 0; i < shapes.size(); ++i) {
        char t[160];
        std::snprintf(t, sizeof(t), "%s[%d, %d, %.3f, %.3f, %.3f, %.3f]", i ? ", " : "", shapes[i].C, shapes[i].nch,
                      shapes[i].ms[0], shapes[i].ms[1], shapes[i].ms[2], shapes[i].ms[3]);
        sh += t;
    }
    sh += "]";
    char fields[128];
    std::snprintf(fields, sizeof(fields), "\": {\"block_nodes\": %d, \"wg_per_cu\": %d, \"shapes\": ", block, wg);
    char ms_field[64];
    std::snprintf(ms_field, sizeof(ms_field), ", \"ms\": %.3f}", ms);
    const std::string entry = "\"" + key + fields + sh + ms_field;
    std::string out;
    if (close == std::string::npos || text.find('{') == std::string::npos) {
        out = "{\n " + entry + "\n}\n";
    } else {
        std::string head = text.substr(0, close);
        while (!head.empty() && (head.back() == '\n' || head.back() == ' ')) head.pop_back();
        out = head + (head.back() == '{' ? "\n " : ",\n ") + entry + "\n}\n";
    }
    if (FILE *f = std::fopen(path, "wb")) {
        std::fwrite(out.data(), 1, out.size(), f);
        std::fclose(f);
    }
}

}  // namespace

extern "C" {

void sq_default_options(sq_options *opt) {
    if (!opt) return;
    opt->precision = SQ_FP64;
    opt->n_lanczos = 50;
    opt->margin = 0.05;
    opt->mu_xtol = 1e-14;
    opt->ne_rtol = 1e-13;
    opt->max_brent = 200;
    opt->workgroups = 0;
}

const char *sq_last_error(void) { return g_error.c_str(); }

int sq_setup(sq_ctx **ctx, double cell, double h, int fd_order, double rcut, int npl, double kT, int natom,
             const double *atom_xyz, const double *kb, const sq_options *opt) {
    return guarded([&]() -> int {
        g_error.clear();
        if (!ctx) return fail(SQ_EINVAL, "ctx is NULL");
        *ctx = nullptr;
        if (!(is_finite(cell) && cell > 0)) return fail(SQ_EINVAL, "cell must be finite and > 0");
        if (!(is_finite(h) && h > 0)) return fail(SQ_EINVAL, "h must be finite and > 0");
        if (fd_order < 2 || fd_order > 2 * sq::kNoMax || (fd_order & 1))
            return fail(SQ_EINVAL, "fd_order must be even in [2, 12]");
        if (!(is_finite(rcut) && rcut > 0)) return fail(SQ_EINVAL, "rcut must be finite and > 0");
        if (npl < 4 || npl > 1000 || npl % 4 != 0) return fail(SQ_EINVAL, "npl must be a multiple of 4 in [4, 1000]");
        if (!(is_finite(kT) && kT > 0)) return fail(SQ_EINVAL, "kT must be finite and > 0");
        if (natom < 0) return fail(SQ_EINVAL, "natom must be >= 0");
        if (natom > 0 && (!atom_xyz || !kb)) return fail(SQ_EINVAL, "atom_xyz and kb are required when natom > 0");
        sq_options o;
        sq_default_options(&o);
        if (opt) o = *opt;
        if (o.precision != SQ_FP64 && o.precision != SQ_FP32_MIXED) return fail(SQ_EINVAL, "unknown precision");
        if (o.n_lanczos < 1 || o.n_lanczos > sq::kMaxLanczos) return fail(SQ_EINVAL, "n_lanczos must be in [1, 256]");
        if (!(is_finite(o.margin) && o.margin >= 0)) return fail(SQ_EINVAL, "margin must be >= 0");
        if (!(o.mu_xtol >= 0) || !(o.ne_rtol >= 0) || o.max_brent < 1)
            return fail(SQ_EINVAL, "invalid Brent tolerances");
        if (o.workgroups < 0) return fail(SQ_EINVAL, "workgroups must be >= 0");

        const double nreal = std::floor(cell / h + 0.5);
        if (nreal < 1 || nreal > 2000) return fail(SQ_EINVAL, "grid must have 1..2000 points per axis");
        auto c = std::unique_ptr<sq_ctx>(new sq_ctx());
        c->cell = cell;
        c->n = int(nreal);
        c->h = cell / c->n;
        c->fd_order = fd_order;
        c->no = fd_order / 2;
        const double mreal = std::floor(rcut / c->h + 0.5);
        if (mreal < 1) return fail(SQ_EINVAL, "R_cut must cover at least one mesh interval (m >= 1)");
        if (mreal > 1000) return fail(SQ_EINVAL, "R_cut too large");
        c->m = int(mreal);
        c->C = 2 * c->m + 1;
        if (c->C > sq::kMaxCube || sq::recurrence_block(c->C) == 0)
            return fail(SQ_EINVAL, "region of influence wider than 37 grid points is not supported");
        c->npl = npl;
        c->nq = npl + 1;
        c->kT = kT;
        c->nd = (long long)c->n * c->n * c->n;
        c->ns = (long long)c->C * c->C * c->C;
        c->opt = o;
        if (c->nd * 8 >= (1LL << 31) || c->ns * 8 >= (1LL << 31))
            return fail(SQ_EINVAL, "grid too large: N_d * 8 bytes must stay below 2 GiB");
        laplacian_weights(c->no, c->h, c->w);

        // one box size for every atom's projector values
        int rbox = 0;
        for (int a = 0; a < natom; ++a) {
            const double rc = kb[3 * a + 1];
            if (is_finite(rc) && rc > 0 && rc / c->h <= 100) rbox = std::max(rbox, sphere_reach(rc, c->h));
        }
        c->pstride = (2 * rbox + 2) * (2 * rbox + 2);
        for (int a = 0; a < natom; ++a) {
            const double *R = atom_xyz + 3 * a;
            const double sig = kb[3 * a], rc = kb[3 * a + 1], gam = kb[3 * a + 2];
            if (!(is_finite(R[0]) && is_finite(R[1]) && is_finite(R[2])))
                return fail(SQ_EINVAL, "non-finite atom position");
            if (!(is_finite(sig) && sig > 0 && is_finite(rc) && rc > 0 && is_finite(gam)))
                return fail(SQ_EINVAL, "projector parameters must be finite with s > 0 and r_c > 0");
            if (rc / c->h > 100) return fail(SQ_EINVAL, "projector cut radius exceeds 100 mesh intervals");
            if (std::fabs(R[0]) / c->h > 1e8 || std::fabs(R[1]) / c->h > 1e8 || std::fabs(R[2]) / c->h > 1e8)
                return fail(SQ_EINVAL, "atom position too far from the cell");
            int rc2 = build_atom_table(c.get(), R, sig, rc, gam, rbox);
            if (rc2) return rc2;
        }
        // deepest overlap of projector spheres at a grid point (periodic count of
        // atom images): the per-column run chains the kernels must carry
        {
            std::vector<int> depth(size_t(c->nd), 0);
            const long long n = c->n;
            auto wrap = [n](long long v) { long long r = v % n; return r < 0 ? r + n : r; };
            for (const auto &at : c->atoms)
                for (int r = 0; r < at.nrun; ++r) {
                    const sq::RunDev &run = c->runs[size_t(at.run0 + r)];
                    const long long gx = wrap(at.bx + run.dx), gy = wrap(at.by + run.dy);
                    for (int k = 0; k < run.len; ++k) {
                        const long long gz = wrap(at.bz + run.dz0 + k);
                        const int d = ++depth[size_t(gx + n * (gy + n * gz))];
                        if (d > c->max_overlap) c->max_overlap = d;
                    }
                }
            if (c->max_overlap > 4)
                return fail(SQ_ECAPACITY, "more than four projector spheres overlap at a grid point");
            if (c->max_overlap > 2 && c->C > sq::kResidentCube)
                return fail(SQ_ECAPACITY, "regions wider than 31 points support at most two overlapping projector spheres");
            c->nch = c->max_overlap > 2 ? 4 : (c->max_overlap > 1 ? 2 : 1);
        }
        // discrete-orthogonality table on N_q = n_pl + 1 Chebyshev-Gauss nodes
        c->ctab.assign(size_t(c->nq) * c->nq, 0.0);
        c->rk.assign(c->nq, 0.0);
        const double pi = 3.14159265358979323846;
        for (int k = 0; k < c->nq; ++k) c->rk[k] = std::cos(pi * (k + 0.5) / c->nq);
        for (int j = 0; j < c->nq; ++j)
            for (int k = 0; k < c->nq; ++k)
                c->ctab[size_t(j) * c->nq + k] = (j == 0 ? 1.0 : 2.0) / c->nq * std::cos(j * pi * (k + 0.5) / c->nq);
        // Lanczos start vector: u(a) - 1/2, u(a) = (SplitMix64(a) >> 11) 2^-53
        double s2 = 0.0;
        for (long long a = 0; a < c->ns; ++a) {
            const double u = double(splitmix64_first(uint64_t(a)) >> 11) * (1.0 / 9007199254740992.0) - 0.5;
            s2 += u * u;
        }
        c->start_norm = std::sqrt(s2);
        int rc = pick_workgroups(c.get());
        if (rc) return rc;
        layout(c.get());
        *ctx = c.release();
        return SQ_OK;
    });
}

int sq_query(const sq_ctx *c, int *n, int *m, long long *n_nodes, size_t *workspace_bytes) {
    if (!c) return fail(SQ_EINVAL, "null context");
    if (n) *n = c->n;
    if (m) *m = c->m;
    if (n_nodes) *n_nodes = c->nd;
    if (workspace_bytes) *workspace_bytes = c->total;
    return SQ_OK;
}

int sq_bind(sq_ctx *c, void *workspace, size_t bytes, const double *veff, void *stream) {
    return guarded([&]() -> int {
        if (!c) return fail(SQ_EINVAL, "null context");
        if (!workspace || !veff) return fail(SQ_EINVAL, "workspace and veff must be device pointers");
        if (bytes < c->total) return fail(SQ_ENOMEM, "workspace smaller than sq_query's workspace_bytes");
        if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(SQ_EINVAL, "workspace must be 256-byte aligned");
        hipStream_t s = static_cast<hipStream_t>(stream);
        c->ws = static_cast<char *>(workspace);
        auto put = [&](size_t off, const void *src, size_t nb) -> int {
            if (nb == 0) return SQ_OK;
            return hip_check(hipMemcpyAsync(c->ws + off, src, nb, hipMemcpyHostToDevice, s), "uploading tables");
        };
        int rc = put(c->off_atoms, c->atoms.data(), c->atoms.size() * sizeof(sq::AtomDev));
        if (!rc) rc = put(c->off_runs, c->runs.data(), c->runs.size() * sizeof(sq::RunDev));
        if (!rc) rc = put(c->off_pvals, c->pvals.data(), c->pvals.size() * sizeof(double));
        if (!rc) rc = put(c->off_ctab, c->ctab.data(), c->ctab.size() * sizeof(double));
        if (!rc) rc = put(c->off_rk, c->rk.data(), c->rk.size() * sizeof(double));
        if (!rc) rc = upload_veff(c, veff, s);
        if (!rc) rc = hip_check(hipStreamSynchronize(s), "binding workspace");
        if (rc) return rc;
        c->state = kBound;
        return SQ_OK;
    });
}

int sq_update_veff(sq_ctx *c, const double *veff, void *stream) {
    int rc = check_ctx(c, kBound);
    if (rc) return rc;
    if (!veff) return fail(SQ_EINVAL, "veff must be a device pointer");
    rc = upload_veff(c, veff, static_cast<hipStream_t>(stream));
    if (rc) return rc;
    c->state = kBound;
    return SQ_OK;
}

int sq_spectral_bounds(sq_ctx *c, double *lmin, double *lmax, void *stream) {
    return guarded([&]() -> int {
        int rc = check_ctx(c, kBound);
        if (rc) return rc;
        hipStream_t s = static_cast<hipStream_t>(stream);
        rc = hip_check(hipMemsetAsync(c->at<int>(c->off_flags), 0, sizeof(int), s), "clearing flags");
        if (rc) return rc;
        sq::RecurrenceArgs a = recurrence_args(c);
        a.lmin = lmin;
        a.lmax = lmax;
        sq::LaunchArgs k;
        rc = stage_launch(c, a, 0, s, &k);
        if (rc) return rc;
        rc = hip_check(sq::launch_lanczos(k, c->C, c->nch, c->nwg_lanczos, s), "launching Lanczos");
        if (rc) return rc;
        ++c->bounds_gen;
        rc = read_flags(c, s);
        if (rc) return rc;
        c->state = kBounds;
        return SQ_OK;
    });
}

int sq_set_bounds(sq_ctx *c, const double *lmin, const double *lmax, void *stream) {
    int rc = check_ctx(c, kBound);
    if (rc) return rc;
    if (!lmin || !lmax) return fail(SQ_EINVAL, "lmin and lmax must be device pointers");
    rc = hip_check(sq::launch_set_bounds(lmin, lmax, c->at<double>(c->off_chi), c->at<double>(c->off_zeta), c->nd,
                                         c->opt.margin, static_cast<hipStream_t>(stream)),
                   "set bounds");
    if (rc) return rc;
    ++c->bounds_gen;
    c->state = kBounds;
    return SQ_OK;
}

int sq_moments(sq_ctx *c, double *moments, void *stream) {
    return guarded([&]() -> int {
        int rc = check_ctx(c, kBounds);
        if (rc) return rc;
        if (!moments) return fail(SQ_EINVAL, "moments must be a device pointer");
        hipStream_t s = static_cast<hipStream_t>(stream);
        rc = hip_check(hipMemsetAsync(c->at<int>(c->off_flags), 0, sizeof(int), s), "clearing flags");
        if (rc) return rc;
        sq::RecurrenceArgs a = recurrence_args(c);
        a.moments = moments;
        sq::LaunchArgs k;
        rc = stage_launch(c, a, 1, s, &k);
        if (rc) return rc;
        rc = hip_check(sq::launch_moments(k, c->C, c->nch, c->opt.precision == SQ_FP32_MIXED, c->nwg_moments, s),
                       "launching moments");
        if (rc) return rc;
        return read_flags(c, s);
    });
}

int sq_fermi_level(sq_ctx *c, const double *moments, double n_electrons, double *mu, void *stream) {
    return guarded([&]() -> int {
        int rc = check_ctx(c, kBounds);
        if (rc) return rc;
        if (!moments || !mu) return fail(SQ_EINVAL, "moments (device) and mu (host) are required");
        if (!(is_finite(n_electrons) && n_electrons > 0 && n_electrons < 2.0 * double(c->nd)))
            return fail(SQ_EINVAL, "n_electrons must lie in (0, 2 N_d)");
        hipStream_t s = static_cast<hipStream_t>(stream);
        rc = hip_check(sq::launch_quadrature_weights(moments, c->at<double>(c->off_ctab), c->at<double>(c->off_W),
                                                     c->nd, c->npl, s),
                       "quadrature weights");
        if (rc) return rc;
        rc = hip_check(sq::launch_extent(c->at<double>(c->off_chi), c->at<double>(c->off_zeta), c->nd,
                                         c->at<double>(c->off_part), kReduceBlocks, c->at<double>(c->off_scal), s),
                       "spectral extent");
        if (rc) return rc;
        double ext[2];
        rc = device_scalars(c, s, ext, 2);
        if (rc) return rc;
        // Brent's method (inverse quadratic interpolation, secant, bisection)
        // on f(mu) = N(mu) - N_e over the spectral bracket; the same state
        // machine runs on the device for batched snapshots.
        sq::BrentState b;
        sq::brent_begin(b, ext[0], ext[1], c->kT, n_electrons, c->opt.mu_xtol, c->opt.ne_rtol * n_electrons,
                        c->opt.max_brent);
        while (b.phase >= sq::kBrentLow && b.phase <= sq::kBrentIterate) {
            double count = 0.0;
            rc = electron_count(c, b.mu_eval, s, &count);
            if (rc) return rc;
            sq::brent_feed(b, count);
        }
        if (b.phase == sq::kBrentDone) {
            *mu = b.xb;
            return SQ_OK;
        }
        if (b.phase == sq::kBrentNonFinite) return fail(SQ_ENOCONV, "non-finite electron count");
        if (b.phase == sq::kBrentNoSign)
            return fail(SQ_ENOCONV, "electron count does not change sign over the spectral bracket");
        return fail(SQ_ENOCONV, "Fermi level search did not converge");
    });
}

int sq_density_energy(sq_ctx *c, const double *moments, double mu, double *rho, double *energies, void *stream) {
    return guarded([&]() -> int {
        int rc = check_ctx(c, kBounds);
        if (rc) return rc;
        if (!moments || !rho || !energies) return fail(SQ_EINVAL, "moments, rho (device) and energies (host) are required");
        if (!is_finite(mu)) return fail(SQ_EINVAL, "mu must be finite");
        hipStream_t s = static_cast<hipStream_t>(stream);
        rc = hip_check(sq::launch_quadrature_weights(moments, c->at<double>(c->off_ctab), c->at<double>(c->off_W),
                                                     c->nd, c->npl, s),
                       "quadrature weights");
        if (rc) return rc;
        const double h3 = c->h * c->h * c->h;
        rc = hip_check(sq::launch_density(c->at<double>(c->off_W), c->at<double>(c->off_chi),
                                          c->at<double>(c->off_zeta), c->at<double>(c->off_rk), c->nd, c->nq, mu,
                                          nullptr, c->kT, h3, rho, c->at<double>(c->off_part), kReduceBlocks,
                                          c->at<double>(c->off_scal), s),
                       "density");
        if (rc) return rc;
        double v[3];
        rc = device_scalars(c, s, v, 3);
        if (rc) return rc;
        energies[0] = v[0];
        energies[1] = v[1];
        energies[2] = v[0] + v[1];
        energies[3] = h3 * v[2];
        return SQ_OK;
    });
}

int sq_density_energy_static(sq_ctx *c, const double *moments, double mu, double *rho, double *energies,
                             void *stream) {
    return guarded([&]() -> int {
        int rc = check_ctx(c, kBounds);
        if (rc) return rc;
        if (!moments || !rho || !energies) return fail(SQ_EINVAL, "moments, rho (device) and energies (host) are required");
        if (!is_finite(mu)) return fail(SQ_EINVAL, "mu must be finite");
        hipStream_t s = static_cast<hipStream_t>(stream);
        double *scratch = nullptr;
        size_t bytes = 0;
        rc = hip_check(sq::static_scratch(&scratch, &bytes), "static scratch address");
        if (rc) return rc;
        // the partials of at most 1024 reduction blocks and three sums: the
        // fixed scratch holds them for any cell size
        if (bytes < sizeof(double) * (3 * 1024 + 4))
            return fail(SQ_ENOMEM, "static scratch smaller than the reduction needs");
        double *sums = nullptr;
        const double h3 = c->h * c->h * c->h;
        rc = hip_check(sq::launch_density_static(moments, c->at<double>(c->off_ctab), c->at<double>(c->off_chi),
                                                 c->at<double>(c->off_zeta), c->at<double>(c->off_rk), c->nd, c->nq,
                                                 mu, c->kT, h3, rho, scratch, &sums, s),
                       "density (static scratch)");
        if (rc) return rc;
        double v[3];
        rc = hip_check(hipMemcpyAsync(v, sums, sizeof(v), hipMemcpyDeviceToHost, s), "reading device sums");
        if (!rc) rc = hip_check(hipStreamSynchronize(s), "density (static scratch)");
        if (rc) return rc;
        energies[0] = v[0];
        energies[1] = v[1];
        energies[2] = v[0] + v[1];
        energies[3] = h3 * v[2];
        return SQ_OK;
    });
}

int sq_nl_forces(sq_ctx *c, double mu, double *forces, void *stream) {
    return guarded([&]() -> int {
        int rc = check_ctx(c, kBounds);
        if (rc) return rc;
        if (!forces) return fail(SQ_EINVAL, "forces must be a host array of natom x 3 doubles");
        if (!is_finite(mu)) return fail(SQ_EINVAL, "mu must be finite");
        if (c->nq > sq::kMaxForceNq) return fail(SQ_EINVAL, "nonlocal forces need n_pl <= 256");
        const size_t na = c->atoms.size();
        for (size_t i = 0; i < 3 * na; ++i) forces[i] = 0.0;
        if (na == 0) return SQ_OK;
        hipStream_t s = static_cast<hipStream_t>(stream);
        double *fdev = c->at<double>(c->off_forces);
        rc = hip_check(sq::launch_zero_doubles(fdev, int(3 * na), s), "clearing forces");
        if (rc) return rc;
        sq::RecurrenceArgs a = recurrence_args(c);
        a.mu = mu;
        a.forces = fdev;
        sq::LaunchArgs k;
        rc = stage_launch(c, a, 1, s, &k);
        if (rc) return rc;
        rc = hip_check(sq::launch_forces(k, c->C, c->nch, c->nwg_lanczos, s), "launching forces");
        if (rc) return rc;
        rc = hip_check(hipMemcpyAsync(forces, fdev, 3 * na * sizeof(double), hipMemcpyDeviceToHost, s),
                       "reading forces");
        if (rc) return rc;
        return hip_check(hipStreamSynchronize(s), "forces");
    });
}

void sq_destroy(sq_ctx *c) { delete c; }

void sq_batch_default_options(sq_batch_options *opt) {
    if (!opt) return;
    opt->block_nodes = 0;
    opt->wg_per_cu = 0;
    opt->use_graph = 1;
    opt->bounds_every = 1;
    opt->reuse_check = 1;
    opt->shape = 0;
}

int sq_batch_create(sq_batch **out, sq_ctx *const *ctxs, int n, double *const *moments, double *const *rho,
                    const double *n_electrons, const sq_batch_options *opt) {
    return guarded([&]() -> int {
        if (!out) return fail(SQ_EINVAL, "batch out pointer is null");
        *out = nullptr;
        if (!ctxs || n < 1) return fail(SQ_EINVAL, "a batch needs n >= 1 contexts");
        if (!moments || !rho || !n_electrons) return fail(SQ_EINVAL, "moments, rho and n_electrons arrays are required");
        auto b = std::unique_ptr<sq_batch>(new sq_batch());
        sq_batch_default_options(&b->opt);
        if (opt) b->opt = *opt;
        if (b->opt.block_nodes < 0 || b->opt.wg_per_cu < 0 || b->opt.bounds_every < 0)
            return fail(SQ_EINVAL, "invalid batch options");
        if (b->opt.block_nodes > 0 && b->opt.block_nodes < 8) return fail(SQ_EINVAL, "block_nodes must be 0 or >= 8");
        if (b->opt.shape & ~(SQ_SHAPE_TWO_ROWS | SQ_SHAPE_TWO_PLANES)) return fail(SQ_EINVAL, "unknown shape bits");
        for (int i = 0; i < n; ++i) {
            sq_ctx *c = ctxs[i];
            int rc = check_ctx(c, kBound);
            if (rc) return rc;
            if (!moments[i] || !rho[i]) return fail(SQ_EINVAL, "moments[i] and rho[i] must be device pointers");
            if (!(is_finite(n_electrons[i]) && n_electrons[i] > 0 && n_electrons[i] < 2.0 * double(c->nd)))
                return fail(SQ_EINVAL, "n_electrons[i] must lie in (0, 2 N_d)");
            const bool mixed = c->opt.precision == SQ_FP32_MIXED;
            if (i == 0) b->mixed = mixed;
            else if (mixed != b->mixed) return fail(SQ_EINVAL, "all contexts of a batch must share one precision");
            if (c->C > sq::kResidentCube && c->nch > 2)
                return fail(SQ_ECAPACITY, "regions wider than 31 points support at most two overlapping projector spheres");
            b->ctx.push_back(c);
            b->moments.push_back(moments[i]);
            b->rho.push_back(rho[i]);
            b->n_e.push_back(n_electrons[i]);
            b->max_brent = i == 0 ? c->opt.max_brent : std::max(b->max_brent, c->opt.max_brent);
            // slots hold the layout of any shape the autotuner may pick
            b->max_slot = std::max({b->max_slot, sq::slot_elems_for(c->C, 0), sq::slot_elems_for(c->C, 1)});
            // one launch per cube side and chain count
            auto g = std::find_if(b->groups.begin(), b->groups.end(),
                                  [&](const sq_batch::Group &x) { return x.C == c->C && x.nch == c->nch; });
            if (g == b->groups.end()) {
                sq_batch::Group ng;
                ng.C = c->C;
                ng.nch = c->nch;
                b->groups.push_back(ng);
                g = b->groups.end() - 1;
            }
            g->snaps.push_back(i);
        }
        int rc = hip_check(hipGetDevice(&b->device), "hipGetDevice");
        if (rc) return rc;
        rc = hip_check(hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device), "CU count");
        if (rc) return rc;
        hipDeviceProp_t prop;
        rc = hip_check(hipGetDeviceProperties(&prop, b->device), "device properties");
        if (rc) return rc;
        std::snprintf(b->device_name, sizeof(b->device_name), "%s", prop.gcnArchName);
        for (auto &g : b->groups) {
            // every shape of the cube side (buffers are sized for the widest grid)
            const int variants = sq::shape_variants(g.C);
            for (int sh = 0; sh < 4; ++sh) {
                if (sh & ~variants) continue;
                rc = hip_check(sq::recurrence_occupancy(g.C, true, false, g.nch, &g.occ_lv[sh], sh),
                               "occupancy (Lanczos)");
                if (!rc)
                    rc = hip_check(sq::recurrence_occupancy(g.C, false, b->mixed, g.nch, &g.occ_mv[sh], sh),
                                   "occupancy (moments)");
                if (rc) return rc;
                if (g.occ_lv[sh] < 1 || g.occ_mv[sh] < 1)
                    return fail(SQ_EDEVICE, "recurrence kernel does not fit on a compute unit");
                b->nwg_cap = std::max({b->nwg_cap, b->cus * g.occ_lv[sh], b->cus * g.occ_mv[sh]});
            }
            g.set_shape(b->opt.shape & variants);
        }
        b->block_nodes = b->opt.block_nodes > 0 ? b->opt.block_nodes : 32;
        b->wg_per_cu = b->opt.wg_per_cu;
        build_items(b.get(), b->block_nodes, 1.0);
        b->args.resize(size_t(n));
        b->fermi.resize(size_t(n));
        b->prm.resize(size_t(n));
        b->state_host.resize(size_t(n));
        b->scal_host.resize(3 * size_t(n));
        b->flags_host.resize(size_t(n));
        for (int i = 0; i < n; ++i) {
            sq_ctx *c = b->ctx[size_t(i)];
            sq::BrentParams &p = b->prm[size_t(i)];
            p.kT = c->kT;
            p.n_e = b->n_e[size_t(i)];
            p.xtol = c->opt.mu_xtol;
            p.ftol = c->opt.ne_rtol * b->n_e[size_t(i)];
            p.max_it = c->opt.max_brent;
        }
        batch_layout(b.get());
        rc = hip_check(hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking), "creating the batch stream");
        if (!rc) rc = hip_check(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming), "creating events");
        if (!rc) rc = hip_check(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming), "creating events");
        if (rc) return rc;
        *out = b.release();
        return SQ_OK;
    });
}

int sq_batch_query(const sq_batch *b, size_t *bytes) {
    if (!b) return fail(SQ_EINVAL, "null batch");
    if (bytes) *bytes = b->total;
    return SQ_OK;
}

int sq_batch_bind(sq_batch *b, void *workspace, size_t bytes, void *stream) {
    return guarded([&]() -> int {
        if (!b) return fail(SQ_EINVAL, "null batch");
        if (!workspace) return fail(SQ_EINVAL, "workspace must be a device pointer");
        if (bytes < b->total) return fail(SQ_ENOMEM, "workspace smaller than sq_batch_query's workspace_bytes");
        if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(SQ_EINVAL, "workspace must be 256-byte aligned");
        hipStream_t s = static_cast<hipStream_t>(stream);
        drop_graph(b);
        b->ws = static_cast<char *>(workspace);
        for (size_t i = 0; i < b->ctx.size(); ++i) {
            sq_ctx *c = b->ctx[i];
            sq::FermiSnap &f = b->fermi[i];
            f.W = c->at<double>(c->off_W);
            f.chi = c->at<double>(c->off_chi);
            f.zeta = c->at<double>(c->off_zeta);
            f.rk = c->at<double>(c->off_rk);
            f.nd = c->nd;
            f.nq = c->nq;
            f.kT = c->kT;
        }
        int rc = hip_check(hipMemcpyAsync(b->at<sq::FermiSnap>(b->off_fermi), b->fermi.data(),
                                          b->fermi.size() * sizeof(sq::FermiSnap), hipMemcpyHostToDevice, s),
                           "uploading batch tables");
        if (!rc)
            rc = hip_check(hipMemcpyAsync(b->at<sq::BrentParams>(b->off_prm), b->prm.data(),
                                          b->prm.size() * sizeof(sq::BrentParams), hipMemcpyHostToDevice, s),
                           "uploading batch tables");
        if (!rc) rc = upload_items(b, s);
        if (!rc) rc = hip_check(hipStreamSynchronize(s), "binding batch workspace");
        return rc;
    });
}

int sq_batch_step(sq_batch *b, double *mu, double *energies, void *stream) {
    return guarded([&]() -> int {
        if (!b) return fail(SQ_EINVAL, "null batch");
        if (!b->ws) return fail(SQ_ESTATE, "call order: sq_batch_bind has not been called");
        for (sq_ctx *c : b->ctx) {
            int rc = check_ctx(c, kBound);
            if (rc) return rc;
        }
        hipStream_t caller = static_cast<hipStream_t>(stream);
        // the pass runs on the batch's own stream (a graph cannot be captured on
        // the null stream), ordered after the caller's work
        int rc = hip_check(hipEventRecord(b->ev_in, caller), "ordering the batch");
        if (!rc) rc = hip_check(hipStreamWaitEvent(b->own, b->ev_in, 0), "ordering the batch");
        if (!rc) rc = upload_args(b, b->own);
        if (rc) return rc;
        // bounds on the first pass, every bounds_every passes, and whenever
        // V_eff has moved too far for the previous ones
        bool bounds = !b->have_bounds || b->opt.bounds_every <= 1 || b->passes % b->opt.bounds_every == 0;
        // bounds rewritten outside the batch since its last pass are not the
        // ones whose margin slack the batch recorded
        for (size_t i = 0; !bounds && i < b->ctx.size(); ++i)
            if (b->ctx[i]->bounds_gen != b->gen_seen[i]) bounds = true;
        if (!bounds && b->opt.reuse_check) {
            bool safe = false;
            rc = reuse_is_safe(b, b->own, &safe);
            if (rc) return rc;
            bounds = !safe;
        }
        auto launch = [&](bool with_bounds) -> int {
            const int g = with_bounds ? 1 : 0;
            if (!b->opt.use_graph) return enqueue_pass(b, with_bounds, b->own);
            if (!b->exec[g]) {
                int r = hip_check(hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal), "graph capture");
                if (r) return r;
                const int rc_pass = enqueue_pass(b, with_bounds, b->own);
                hipGraph_t gr = nullptr;
                const int rc_end = hip_check(hipStreamEndCapture(b->own, &gr), "graph capture");
                if (rc_pass || rc_end) {
                    if (gr) (void)hipGraphDestroy(gr);
                    return rc_pass ? rc_pass : rc_end;
                }
                b->graph[g] = gr;
                r = hip_check(hipGraphInstantiate(&b->exec[g], gr, nullptr, nullptr, 0), "graph instantiation");
                if (r) {
                    (void)hipGraphDestroy(gr);
                    b->graph[g] = nullptr;
                    b->exec[g] = nullptr;
                    return r;
                }
            }
            return hip_check(hipGraphLaunch(b->exec[g], b->own), "graph launch");
        };
        rc = launch(bounds);
        if (rc) return rc;
        rc = finish_pass(b, b->own, mu, energies);
        if (rc == SQ_EBOUNDS && !bounds) {
            // reused bounds no longer enclose a spectrum: redo with fresh ones
            bounds = true;
            rc = launch(true);
            if (!rc) rc = finish_pass(b, b->own, mu, energies);
        }
        if (!rc && bounds && b->opt.bounds_every > 1) rc = record_bounds(b, b->own);
        if (!rc) {
            ++b->passes;
            b->have_bounds = true;
            b->gen_seen.resize(b->ctx.size());
            for (size_t i = 0; i < b->ctx.size(); ++i) {
                if (bounds) ++b->ctx[i]->bounds_gen;
                b->gen_seen[i] = b->ctx[i]->bounds_gen;
            }
        }
        const int rc2 = hip_check(hipEventRecord(b->ev_out, b->own), "ordering the batch");
        if (!rc2) (void)hipStreamWaitEvent(caller, b->ev_out, 0);
        return rc ? rc : rc2;
    });
}

int sq_batch_autotune(sq_batch *b, const char *cache_path, void *stream) {
    return guarded([&]() -> int {
        if (!b) return fail(SQ_EINVAL, "null batch");
        if (!b->ws) return fail(SQ_ESTATE, "call order: sq_batch_bind has not been called");
        hipStream_t caller = static_cast<hipStream_t>(stream);
        int rc = hip_check(hipStreamSynchronize(caller), "autotune");
        if (rc) return rc;
        drop_graph(b);
        b->have_bounds = false;  // the tuning runs rewrite chi and zeta
        const std::string key = tune_key(b);
        int best_block = 0, best_wg = 0;
        std::vector<TunedShape> shapes;
        if (!cache_lookup(cache_path, key, &best_block, &best_wg, &shapes)) {
            shapes.clear();
            rc = upload_args(b, b->own);
            if (rc) return rc;
            for (auto &g : b->groups) g.set_shape(0);
            int max_occ = 1;
            for (const auto &g : b->groups) max_occ = std::max({max_occ, g.occ_l, g.occ_m});
            std::vector<int> wgs = {1};
            if (max_occ > 1) wgs.push_back(max_occ);
            hipEvent_t e0, e1;
            rc = hip_check(hipEventCreate(&e0), "autotune events");
            if (!rc) rc = hip_check(hipEventCreate(&e1), "autotune events");
            if (rc) return rc;
            // one timed pass of the sample (only >= 0: that launch group alone)
            auto timed = [&](int only, float *ms) -> int {
                int r = hip_check(hipEventRecord(e0, b->own), "autotune timing");
                if (!r) r = enqueue_recurrences(b, true, true, b->own, only);
                if (!r) r = hip_check(hipEventRecord(e1, b->own), "autotune timing");
                if (!r) r = hip_check(hipEventSynchronize(e1), "autotune timing");
                if (!r) r = hip_check(hipEventElapsedTime(ms, e0, e1), "autotune timing");
                return r;
            };
            double best_ms = 1e300;
            // a sample of every snapshot (its first 1/8 of the nodes) through
            // both recurrence kernels: Lanczos (which also gives the sample's
            // bounds) and the moments, at the default kernel shapes
            for (int block : {8, 32, 128}) {
                for (int wg : wgs) {
                    build_items(b, block, 0.125);
                    b->wg_per_cu = wg;
                    rc = upload_items(b, b->own);
                    float ms = 0.f;
                    if (!rc) rc = timed(-1, &ms);
                    if (rc) break;
                    if (ms < best_ms) {
                        best_ms = ms;
                        best_block = block;
                        best_wg = wg;
                    }
                }
                if (rc) break;
            }
            // then, at that tile, every kernel shape of each group's cube side,
            // the group alone (best of two runs: the first launch of a shape
            // may also load its code object)
            if (!rc) {
                build_items(b, best_block, 0.125);
                b->wg_per_cu = best_wg;
                rc = upload_items(b, b->own);
            }
            for (int gi = 0; !rc && gi < int(b->groups.size()); ++gi) {
                auto &g = b->groups[size_t(gi)];
                const int variants = sq::shape_variants(g.C);
                if (variants == 0 || g.n_items == 0) continue;
                TunedShape t{g.C, g.nch, 0, {-1.0, -1.0, -1.0, -1.0}};
                double best_g = 1e300;
                for (int sh = 0; sh < 4 && !rc; ++sh) {
                    if (sh & ~variants) continue;
                    g.set_shape(sh);
                    float ms = 0.f, ms2 = 0.f;
                    rc = timed(gi, &ms);
                    if (!rc) rc = timed(gi, &ms2);
                    t.ms[sh] = std::min(ms, ms2);
                    if (!rc && t.ms[sh] < best_g) {
                        best_g = t.ms[sh];
                        t.shape = sh;
                    }
                }
                g.set_shape(t.shape);
                shapes.push_back(t);
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            if (rc) return rc;
            cache_store(cache_path, key, best_block, best_wg, shapes, best_ms);
        } else {
            for (auto &g : b->groups) {
                int sh = 0;
                for (const auto &t : shapes)
                    if (t.C == g.C && t.nch == g.nch) sh = t.shape & sq::shape_variants(g.C);
                g.set_shape(sh);
            }
        }
        b->block_nodes = best_block;
        b->wg_per_cu = best_wg;
        build_items(b, b->block_nodes, 1.0);
        rc = upload_items(b, b->own);
        if (!rc) rc = hip_check(hipStreamSynchronize(b->own), "autotune");
        return rc;
    });
}

int sq_batch_tiles(const sq_batch *b, int *block_nodes, int *wg_per_cu, int *n_items) {
    if (!b) return fail(SQ_EINVAL, "null batch");
    if (block_nodes) *block_nodes = b->block_nodes;
    if (wg_per_cu) *wg_per_cu = b->wg_per_cu;
    if (n_items) *n_items = int(b->items.size());
    return SQ_OK;
}

int sq_batch_group(const sq_batch *b, int i, int *cube, int *nch, int *shape, int *n_groups) {
    if (!b) return fail(SQ_EINVAL, "null batch");
    if (n_groups) *n_groups = int(b->groups.size());
    if (i < 0) return SQ_OK;
    if (i >= int(b->groups.size())) return fail(SQ_EINVAL, "launch group index out of range");
    const auto &g = b->groups[size_t(i)];
    if (cube) *cube = g.C;
    if (nch) *nch = g.nch;
    if (shape) *shape = g.shape;
    return SQ_OK;
}

void sq_batch_destroy(sq_batch *b) { delete b; }

}  // extern "C"
