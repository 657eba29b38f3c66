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
    int max_overlap = 0;
    size_t off_atoms = 0, off_runs = 0, off_pvals = 0, off_chi = 0, off_zeta = 0, off_ctab = 0,
           off_rk = 0, off_W = 0, off_part = 0, off_scal = 0, off_flags = 0, off_v32 = 0,
           off_slots = 0, off_wslots = 0, total = 0;
    char *ws = nullptr;
    const double *veff = nullptr;
    int state = kSetup;

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

// Projector of one atom as z-runs over (dx, dy) columns of its sphere.
int build_atom_table(sq_ctx *c, const double *R, double sig, double rc, double gamma) {
    const double h = c->h;
    const int b[3] = {int(std::floor(R[0] / h)), int(std::floor(R[1] / h)), int(std::floor(R[2] / h))};
    const int r = int(std::ceil(rc / h)) + 1;
    const double rc2 = rc * rc;
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
                    c->pvals.push_back(std::exp(-r2 / (2.0 * sig * sig)));
                }
            }
            if (count == 0) continue;
            if (count > 255) return fail(SQ_EINVAL, "projector radius too large for the mesh");
            sq::RunDev run{};
            run.dx = int8_t(dx);
            run.dy = int8_t(dy);
            run.dz0 = int8_t(first);
            run.len = uint8_t(count);
            run.vstart = int32_t(c->pvals.size() - count);
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
    // normalise on the grid: h^3 sum chi^2 = 1 over the whole sphere
    double ss = 0.0;
    for (size_t i = v0; i < c->pvals.size(); ++i) ss += c->pvals[i] * c->pvals[i];
    const double norm = std::sqrt(h * h * h * ss);
    for (size_t i = v0; i < c->pvals.size(); ++i) c->pvals[i] /= norm;
    at.coef = gamma * h * h * h;
    c->atoms.push_back(at);
    if (c->pvals.size() > size_t(std::numeric_limits<int32_t>::max() / 2))
        return fail(SQ_EINVAL, "projector tables too large");
    return SQ_OK;
}

int hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return SQ_OK;
    return fail(SQ_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int read_flags(sq_ctx *c, hipStream_t s) {
    int flags = 0;
    int rc = hip_check(hipMemcpyAsync(&flags, c->at<int>(c->off_flags), sizeof(int), hipMemcpyDeviceToHost, s),
                       "reading device flags");
    if (rc) return rc;
    rc = hip_check(hipStreamSynchronize(s), "kernel execution");
    if (rc) return rc;
    if (flags & sq::kFlagImages) return fail(SQ_ECAPACITY, "more projector images in a region than supported");
    if (flags & sq::kFlagRuns) return fail(SQ_ECAPACITY, "projector run table of a region overflowed");
    if (flags & sq::kFlagOverlap) return fail(SQ_ECAPACITY, "more than two projector spheres overlap");
    if (flags & sq::kFlagLanczos) return fail(SQ_EINVAL, "non-finite Lanczos coefficient (check V_eff)");
    if (flags & sq::kFlagBounds) return fail(SQ_EBOUNDS, "a Chebyshev moment left [-1, 1]: bounds too tight");
    return SQ_OK;
}

sq::RecurrenceArgs recurrence_args(sq_ctx *c) {
    sq::RecurrenceArgs a{};
    a.n = c->n;
    a.m = c->m;
    a.C = c->C;
    a.nd = c->nd;
    for (int d = 0; d <= sq::kNoMax; ++d) a.w[d] = c->w[d];
    a.veff = c->veff;
    a.veff32 = c->opt.precision == SQ_FP32_MIXED ? c->at<float>(c->off_v32) : nullptr;
    a.natom = int(c->atoms.size());
    a.atoms = c->at<sq::AtomDev>(c->off_atoms);
    a.runs = c->at<sq::RunDev>(c->off_runs);
    a.pvals = c->at<double>(c->off_pvals);
    a.pvals_bytes = (long long)(c->pvals.size() * sizeof(double));
    a.chi = c->at<double>(c->off_chi);
    a.zeta = c->at<double>(c->off_zeta);
    a.npl = c->npl;
    a.slots = c->ws + c->off_slots;
    a.wslots = c->ws + c->off_wslots;
    a.slot_elems = c->ns;
    a.flags = c->at<int>(c->off_flags);
    a.nch = c->nch;
    a.n_lanczos = c->opt.n_lanczos;
    a.start_norm = c->start_norm;
    a.margin = c->opt.margin;
    a.bounds_tol = c->opt.precision == SQ_FP32_MIXED ? 1e-5 : 1e-10;
    return a;
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
    c->off_v32 = take(c->opt.precision == SQ_FP32_MIXED ? size_t(c->nd) * sizeof(float) : 0);
    c->off_slots = take(size_t(c->nwg_slots) * size_t(c->ns) * sizeof(double));
    c->off_wslots = take(size_t(c->nwg_lanczos) * size_t(c->ns) * sizeof(double));
    c->total = off;
}

int upload_veff(sq_ctx *c, const double *veff, hipStream_t s) {
    c->veff = veff;
    if (c->opt.precision == SQ_FP32_MIXED) {
        int rc = hip_check(sq::launch_to_fp32(veff, c->at<float>(c->off_v32), c->nd, s), "V_eff to FP32");
        if (rc) return rc;
    }
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
            return fail(SQ_EINVAL, "region of influence wider than 31 grid points is not supported");
        c->npl = npl;
        c->nq = npl + 1;
        c->kT = kT;
        c->nd = (long long)c->n * c->n * c->n;
        c->ns = (long long)c->C * c->C * c->C;
        c->opt = o;
        if (c->nd * 8 >= (1LL << 31) || c->ns * 8 >= (1LL << 31))
            return fail(SQ_EINVAL, "grid too large: N_d * 8 bytes must stay below 2 GiB");
        laplacian_weights(c->no, c->h, c->w);

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
            int rc2 = build_atom_table(c.get(), R, sig, rc, gam);
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
            c->nch = c->max_overlap > 2 ? 4 : 2;
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
        rc = hip_check(sq::launch_lanczos(a, c->nwg_lanczos, s), "launching Lanczos");
        if (rc) return rc;
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
        rc = hip_check(sq::launch_moments(a, c->opt.precision == SQ_FP32_MIXED, c->nwg_moments, s),
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
        // on f(mu) = N(mu) - N_e over the spectral bracket.
        double xa = ext[0] - 40.0 * c->kT, xb = ext[1] + 40.0 * c->kT;
        double fa, fb;
        rc = electron_count(c, xa, s, &fa);
        if (rc) return rc;
        rc = electron_count(c, xb, s, &fb);
        if (rc) return rc;
        fa -= n_electrons;
        fb -= n_electrons;
        if (!(is_finite(fa) && is_finite(fb))) return fail(SQ_ENOCONV, "non-finite electron count");
        if ((fa > 0) == (fb > 0) && fa != 0 && fb != 0)
            return fail(SQ_ENOCONV, "electron count does not change sign over the spectral bracket");
        const double ftol = c->opt.ne_rtol * n_electrons;
        double xc = xa, fc = fa, step = xb - xa, prev_step = step;
        for (int it = 0; it < c->opt.max_brent; ++it) {
            if ((fb > 0 && fc > 0) || (fb < 0 && fc < 0)) {  // keep the root between xb and xc
                xc = xa;
                fc = fa;
                step = prev_step = xb - xa;
            }
            if (std::fabs(fc) < std::fabs(fb)) {  // xb is the best estimate
                xa = xb; xb = xc; xc = xa;
                fa = fb; fb = fc; fc = fa;
            }
            const double tol = 2.0 * std::numeric_limits<double>::epsilon() * std::fabs(xb) + 0.5 * c->opt.mu_xtol;
            const double half = 0.5 * (xc - xb);
            if (std::fabs(half) <= tol || std::fabs(fb) <= ftol || fb == 0.0) {
                *mu = xb;
                return SQ_OK;
            }
            if (std::fabs(prev_step) >= tol && std::fabs(fa) > std::fabs(fb)) {
                const double sb = fb / fa;
                double p, q;
                if (xa == xc) {  // secant
                    p = 2.0 * half * sb;
                    q = 1.0 - sb;
                } else {  // inverse quadratic interpolation
                    const double qa = fa / fc, rb = fb / fc;
                    p = sb * (2.0 * half * qa * (qa - rb) - (xb - xa) * (rb - 1.0));
                    q = (qa - 1.0) * (rb - 1.0) * (sb - 1.0);
                }
                if (p > 0) q = -q;
                else p = -p;
                if (2.0 * p < 3.0 * half * q - std::fabs(tol * q) && p < std::fabs(0.5 * prev_step * q)) {
                    prev_step = step;
                    step = p / q;
                } else {
                    step = half;
                    prev_step = step;
                }
            } else {
                step = half;
                prev_step = step;
            }
            xa = xb;
            fa = fb;
            xb += std::fabs(step) > tol ? step : (half > 0 ? tol : -tol);
            rc = electron_count(c, xb, s, &fb);
            if (rc) return rc;
            fb -= n_electrons;
        }
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
                                          c->kT, h3, rho, c->at<double>(c->off_part), kReduceBlocks,
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

void sq_destroy(sq_ctx *c) { delete c; }

}  // extern "C"
