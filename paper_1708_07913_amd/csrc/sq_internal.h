// Internal declarations shared by the host side (sq_api.cpp) and the HIP
// kernels (sq_kernels.hip) of libsq.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace sq {

constexpr int kNoMax = 6;        // largest FD half-order (fd_order 12)
constexpr int kMaxImages = 256;  // projector images per region of influence
constexpr int kMaxLanczos = 256; // Lanczos steps per node
constexpr int kMaxCube = 31;     // largest cube side with one column per thread

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
    int32_t vstart;  // index of the dz0 value in the flat value array
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
    const float *veff32;    // n^3 FP32 copy (mixed precision)
    int natom;
    const AtomDev *atoms;
    const RunDev *runs;
    const double *pvals;
    long long pvals_bytes;
    double *chi, *zeta;     // per node
    double *lmin, *lmax;    // Lanczos outputs (may be null)
    double *moments;        // N_d x (npl + 1)
    int npl;
    void *slots;            // nwg slots of C^3 elements
    void *wslots;           // second set of slots (Lanczos: H v - beta v_prev)
    long long slot_elems;
    int *flags;
    int nch;                // projector chains per column: 2 or 4 (max sphere overlap depth)
    int n_lanczos;
    double start_norm;      // norm of the unnormalised Lanczos start vector
    double margin;
    double bounds_tol;      // allowed |moment| - 1
};

// Launchers (sq_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_lanczos(const RecurrenceArgs &a, int nwg, hipStream_t s);
hipError_t launch_moments(const RecurrenceArgs &a, bool mixed, int nwg, hipStream_t s);
int recurrence_block(int C);
hipError_t recurrence_occupancy(int C, bool lanczos, bool mixed, int nch, int *blocks_per_cu);
hipError_t launch_set_bounds(const double *lmin, const double *lmax, double *chi, double *zeta,
                             long long nd, double margin, hipStream_t s);
hipError_t launch_to_fp32(const double *src, float *dst, long long n, hipStream_t s);
hipError_t launch_quadrature_weights(const double *mom, const double *ctab, double *W,
                                     long long nd, int npl, hipStream_t s);
hipError_t launch_extent(const double *chi, const double *zeta, long long nd, double *partials,
                         int nblk, double *out, hipStream_t s);
hipError_t launch_count(const double *W, const double *chi, const double *zeta, const double *rk,
                        long long nd, int nq, double mu, double kT, double *partials, int nblk,
                        double *out, hipStream_t s);
hipError_t launch_density(const double *W, const double *chi, const double *zeta, const double *rk,
                          long long nd, int nq, double mu, double kT, double h3, double *rho,
                          double *partials, int nblk, double *out, hipStream_t s);

}  // namespace sq
