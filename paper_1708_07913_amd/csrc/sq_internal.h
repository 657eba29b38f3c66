// Internal declarations shared by the host side (sq_api.cpp) and the HIP
// kernels (sq_kernels.hip) of libsq.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>

namespace sq {

constexpr int kNoMax = 6;        // largest FD half-order (fd_order 12)
constexpr int kMaxImages = 256;  // projector images per region of influence
constexpr int kMaxLanczos = 256; // Lanczos steps per node
constexpr int kMaxCube = 37;     // largest cube side (region of influence)
constexpr int kResidentCube = 31; // largest cube side whose columns stay in registers

// Rows of the cube owned by one thread of the recurrence kernels: one column
// up to 27 points (a workgroup of C^2 threads, 7-12 waves for 21-27 points),
// two y-adjacent columns for 29 and 31 points (512-thread workgroups, 256
// VGPRs per lane; the pair shares its y-neighbour reads), three beyond 31
// points.  One row on 29 points spills.  The 21-27-point cubes also have a
// two-row shape (`two` = 1: 32-lane row groups, 6-7 waves), built as a
// separate set of kernels that batches may select (kShapeTwoRows).
constexpr bool has_two_row_shape(int C) { return C >= 21 && C <= 27; }
constexpr int rows_per_thread(int C, int two = 0) {
    return C > kResidentCube ? 3 : (C >= 29 || (two && has_two_row_shape(C)) ? 2 : 1);
}
// Threads per row group (lanes along x): two-row shapes give each row group
// 32 lanes, the last ones idle.
constexpr int row_group_threads(int C, int two = 0) {
    return (C == 29 || C == 31 || (two && has_two_row_shape(C))) ? 32 : C;
}
// Doubles per plane of a workgroup's recurrence slot.  The Lanczos ring
// kernel (cubes up to kResidentCube) stores plane z of a vector thread by
// thread: the thread at x in row group g keeps its rows r at elements
// z * slot_plane + (g * C + x) * rows + r, so that it moves all its rows with
// one 8- or 16-byte access and a row group's stores are contiguous.  The
// moments kernels and the streamed kernels store the cube's plane, element
// z * C^2 + y * C + x, which fits as slot_plane >= C^2.
constexpr long long slot_plane(int C, int two = 0) {
    return C > kResidentCube ? (long long)C * C
                             : (long long)((C + rows_per_thread(C, two) - 1) / rows_per_thread(C, two)) * C *
                                   rows_per_thread(C, two);
}
constexpr long long slot_elems_for(int C, int two = 0) { return (long long)C * slot_plane(C, two); }

// Kernel shape variants of the register-ring recurrence kernels (bit set):
// two rows per thread (cubes with has_two_row_shape) and two planes per
// barrier in the FP64 Lanczos and moments sweeps (ring cubes of 21 points
// and more; four LDS plane buffers instead of two).
constexpr int kShapeTwoRows = 1;
constexpr int kShapeTwoPlanes = 2;
constexpr bool has_two_plane_shape(int C) { return C >= 21 && C <= kResidentCube; }
// Variants that exist for cube side C (a subset of the bits above).
constexpr int shape_variants(int C) {
    return (has_two_row_shape(C) ? kShapeTwoRows : 0) | (has_two_plane_shape(C) ? kShapeTwoPlanes : 0);
}

// One atom's projector, stored as z-runs: for every (dx, dy) column of the
// sphere relative to the base node (bx, by, bz) = floor(R / h), the contiguous
// range dz0 .. dz0 + len - 1 of grid points inside the sphere.
struct AtomDev {
    int bx, by, bz;
    int run0, nrun;
    int dmin[3], dmax[3];
    double coef;  // gamma * h^3 (trapezoid rule)
};

struct RunDev {
    int8_t dx, dy, dz0;
    uint8_t len;
    int32_t vstart;  // index of the dz0 value in the flat value array (values of the
                     // run's later planes follow at strides of RecurrenceArgs::pstride)
};

enum Flags : int {
    kFlagImages = 1,    // more than kMaxImages images in a region
    kFlagRuns = 2,      // more projector runs than the per-node table holds
    kFlagOverlap = 4,   // more projector spheres overlap at a point than chains exist
    kFlagBounds = 8,    // a moment left [-1, 1]
    kFlagLanczos = 16,  // non-finite Lanczos coefficient
};

struct RecurrenceArgs {
    int n, m, C;
    long long nd;
    double w[kNoMax + 1];   // FD Laplacian weights w_0..w_6 (zero beyond n_o)
    const double *veff;     // n^3 FP64
    int natom;
    const AtomDev *atoms;
    const RunDev *runs;
    const double *pvals;    // per-atom boxes of projector values, x fastest
    long long pvals_bytes;
    int pstride;            // doubles from a projector value to the one a plane above
    double *chi, *zeta;     // per node
    double *lmin, *lmax;    // Lanczos outputs (may be null)
    double *moments;        // N_d x (npl + 1)
    int npl;
    int *flags;
    int nch;                // projector chains per column: 2 or 4 (max sphere overlap depth)
    int n_lanczos;
    double start_norm;      // norm of the unnormalised Lanczos start vector
    double margin;
    double bounds_tol;      // allowed |moment| - 1
    // nonlocal forces (Sec. 3.4)
    double gw[kNoMax + 1];  // FD gradient weights (zero beyond n_o)
    const double *ctab;     // (n_pl + 1)^2 coefficient table, [j][k]
    const double *rk;       // n_pl + 1 Chebyshev-Gauss nodes
    double mu, kT;          // Fermi level, smearing (Ha)
    double *forces;         // natom x 3, accumulated
};

constexpr int kMaxForceNq = 257;  // n_pl + 1 limit of the force kernel

// One unit of a work queue: nodes q0 .. q1 - 1 of snapshot `snap`.
struct WorkItem {
    int snap;
    int reserved;
    long long q0, q1;
};

// What a recurrence launch works on.  With items == nullptr the launch covers
// every node of snaps[0], split statically over the XCDs; otherwise each
// workgroup takes items from the queue (counter must be zero at launch).
struct LaunchArgs {
    const RecurrenceArgs *snaps;  // device array, read-only during the launch
    const WorkItem *items;        // device array or nullptr
    int n_items;
    int *counter;                 // device work-queue head
    void *slots, *wslots, *xslots;  // per-workgroup vector buffers
    long long slot_elems;         // elements per workgroup buffer (largest N_s of the launch)
};

// ---------------------------------------------------------------------------
// Brent's method for the Fermi level (Sec. 3.2: N(mu) = N_e), written as a
// state machine fed one electron count at a time, so that the host loop and
// the device step kernel of batched snapshots run the same arithmetic.
// ---------------------------------------------------------------------------
#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)
#define SQ_HD __host__ __device__
#else
#define SQ_HD
#endif

enum BrentPhase : int {
    kBrentLow = 0,        // N(lower bracket end) pending
    kBrentHigh = 1,       // N(upper bracket end) pending
    kBrentIterate = 2,    // N(new estimate) pending
    kBrentDone = 3,       // converged; mu = xb
    kBrentNonFinite = -1, // a count was not finite
    kBrentNoSign = -2,    // N - N_e does not change sign over the bracket
    kBrentMaxIt = -3,     // iteration limit reached
};

struct BrentState {
    double xa, xb, xc, fa, fb, fc, step, prev_step;
    double mu_eval;              // where the next count is to be taken
    double n_e, xtol, ftol;      // target, bracket half-width and |N - N_e| tolerances
    int phase, it, max_it, pad;
};

// Bracket [ext_lo - 40 kT, ext_hi + 40 kT] around the scaled spectra of all nodes.
SQ_HD inline void brent_begin(BrentState &b, double ext_lo, double ext_hi, double kT, double n_e, double xtol,
                              double ftol, int max_it) {
#ifdef __clang__
#pragma clang fp contract(off)
#endif
    const double lo = ext_lo - 40.0 * kT, hi = ext_hi + 40.0 * kT;
    b.xa = lo;
    b.xb = hi;
    b.xc = lo;
    b.fa = b.fb = b.fc = 0.0;
    b.step = b.prev_step = hi - lo;
    b.mu_eval = lo;
    b.n_e = n_e;
    b.xtol = xtol;
    b.ftol = ftol;
    b.phase = kBrentLow;
    b.it = 0;
    b.max_it = max_it;
    b.pad = 0;
}

// Feed N(mu_eval).  Afterwards either phase is pending again with a new
// mu_eval, or it is kBrentDone (mu = xb) or an error.
SQ_HD inline void brent_feed(BrentState &b, double count) {
#ifdef __clang__
#pragma clang fp contract(off)
#endif
    const double f = count - b.n_e;
    const bool finite_f = f == f && f - f == 0.0;
    if (b.phase == kBrentLow) {
        b.fa = f;
        b.mu_eval = b.xb;
        b.phase = kBrentHigh;
        return;
    }
    if (b.phase == kBrentHigh) {
        b.fb = f;
        if (!(b.fa == b.fa && b.fa - b.fa == 0.0) || !finite_f) {
            b.phase = kBrentNonFinite;
            return;
        }
        if ((b.fa > 0) == (b.fb > 0) && b.fa != 0 && b.fb != 0) {
            b.phase = kBrentNoSign;
            return;
        }
        b.xc = b.xa;
        b.fc = b.fa;
        b.step = b.prev_step = b.xb - b.xa;
    } else if (b.phase == kBrentIterate) {
        b.fb = f;
        if (!finite_f) {
            b.phase = kBrentNonFinite;
            return;
        }
    } else {
        return;
    }
    if (b.it >= b.max_it) {
        b.phase = kBrentMaxIt;
        return;
    }
    ++b.it;
    if ((b.fb > 0 && b.fc > 0) || (b.fb < 0 && b.fc < 0)) {  // keep the root between xb and xc
        b.xc = b.xa;
        b.fc = b.fa;
        b.step = b.prev_step = b.xb - b.xa;
    }
    if (fabs(b.fc) < fabs(b.fb)) {  // xb is the best estimate
        b.xa = b.xb;
        b.xb = b.xc;
        b.xc = b.xa;
        b.fa = b.fb;
        b.fb = b.fc;
        b.fc = b.fa;
    }
    const double tol = 2.0 * 2.220446049250313e-16 * fabs(b.xb) + 0.5 * b.xtol;
    const double half = 0.5 * (b.xc - b.xb);
    if (fabs(half) <= tol || fabs(b.fb) <= b.ftol || b.fb == 0.0) {
        b.phase = kBrentDone;
        return;
    }
    if (fabs(b.prev_step) >= tol && fabs(b.fa) > fabs(b.fb)) {
        const double sb = b.fb / b.fa;
        double p, q;
        if (b.xa == b.xc) {  // secant
            p = 2.0 * half * sb;
            q = 1.0 - sb;
        } else {  // inverse quadratic interpolation
            const double qa = b.fa / b.fc, rb = b.fb / b.fc;
            p = sb * (2.0 * half * qa * (qa - rb) - (b.xb - b.xa) * (rb - 1.0));
            q = (qa - 1.0) * (rb - 1.0) * (sb - 1.0);
        }
        if (p > 0) q = -q;
        else p = -p;
        if (2.0 * p < 3.0 * half * q - fabs(tol * q) && p < fabs(0.5 * b.prev_step * q)) {
            b.prev_step = b.step;
            b.step = p / q;
        } else {
            b.step = half;
            b.prev_step = b.step;
        }
    } else {
        b.step = half;
        b.prev_step = b.step;
    }
    b.xa = b.xb;
    b.fa = b.fb;
    b.xb += fabs(b.step) > tol ? b.step : (half > 0 ? tol : -tol);
    b.mu_eval = b.xb;
    b.phase = kBrentIterate;
}

// Per-snapshot inputs of the batched electron count.
struct FermiSnap {
    const double *W, *chi, *zeta, *rk;
    long long nd;
    int nq, pad;
    double kT;
};

// Launchers (sq_kernels.hip).  Return hipSuccess or the launch error.
// C is the cube side and nch the projector chains of every snapshot launched.
// `shape`: kShape* bits (0 = the default shape); bits that cube side C does
// not have return hipErrorInvalidValue.
hipError_t launch_lanczos(const LaunchArgs &k, int C, int nch, int nwg, hipStream_t s, int shape = 0);
hipError_t launch_moments(const LaunchArgs &k, int C, int nch, bool mixed, int nwg, hipStream_t s, int shape = 0);
hipError_t launch_forces(const LaunchArgs &k, int C, int nch, int nwg, hipStream_t s);
hipError_t launch_zero_ints(int *p, int n, hipStream_t s);
hipError_t launch_zero_doubles(double *p, int n, hipStream_t s);
int recurrence_block(int C, int shape = 0);
hipError_t recurrence_occupancy(int C, bool lanczos, bool mixed, int nch, int *blocks_per_cu, int shape = 0);
hipError_t launch_set_bounds(const double *lmin, const double *lmax, double *chi, double *zeta,
                             long long nd, double margin, hipStream_t s);
hipError_t launch_quadrature_weights(const double *mom, const double *ctab, double *W,
                                     long long nd, int npl, hipStream_t s);
hipError_t launch_extent(const double *chi, const double *zeta, long long nd, double *partials,
                         int nblk, double *out, hipStream_t s);
// out[0..1] = min, max of a - b over n entries (b may be null: of a).
hipError_t launch_diff_extent(const double *a, const double *b, long long n, double *partials, int nblk,
                              double *out, hipStream_t s);
hipError_t launch_count(const double *W, const double *chi, const double *zeta, const double *rk,
                        long long nd, int nq, double mu, double kT, double *partials, int nblk,
                        double *out, hipStream_t s);
// mu_dev: if not null, mu is read from it (device) instead of `mu`.
hipError_t launch_density(const double *W, const double *chi, const double *zeta, const double *rk,
                          long long nd, int nq, double mu, const double *mu_dev, double kT, double h3,
                          double *rho, double *partials, int nblk, double *out, hipStream_t s);
// Allocation-free density and energies: kernels use the library's static
// device scratch (static_scratch: its device address on the current device,
// looked up once per device, and its size).  *sums receives the device address
// of {sum E_band terms, sum E_ent terms, sum rho}.
constexpr int kMaxDevices = 64;
hipError_t static_scratch(double **ptr, size_t *bytes);
hipError_t launch_density_static(const double *mom, const double *ctab, const double *chi, const double *zeta,
                                 const double *rk, long long nd, int nq, double mu, double kT, double h3,
                                 double *rho, double *scratch_ptr, double **sums, hipStream_t s);
// Batched Fermi level: N(mu_eval) of every snapshot still iterating (grid
// nblk x nsnap, the same per-snapshot partial sums as launch_count), then one
// Brent step per snapshot.
struct BrentParams {
    double kT, n_e, xtol, ftol;
    int max_it, pad;
};
hipError_t launch_brent_begin(BrentState *st, const BrentParams *prm, const double *ext, int nsnap, hipStream_t s);
hipError_t launch_count_batch(const FermiSnap *fs, const BrentState *st, int nsnap, double *partials, int nblk,
                              hipStream_t s);
hipError_t launch_brent_feed(BrentState *st, const double *partials, int nblk, int nsnap, hipStream_t s);

}  // namespace sq
